// C ABI (include/nnp.h): model creation, workspace, and the stage order of
// one energy/force evaluation.  Host code only orchestrates: every step of
// the path runs in the library's kernels on the caller's stream.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/nnp.h"

#include "internal.h"

using namespace nnp;

namespace nnp {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace nnp

namespace {

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(NNP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

// A device buffer that only grows.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return NNP_OK;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return fail(NNP_EDEVICE, "hipFree: %s", hipGetErrorString(e));
      p = nullptr;
      bytes = 0;
    }
    size_t nb = need + need / 4 + 256;
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(NNP_ENOMEM, "hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
    }
    bytes = nb;
    return NNP_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T *as() const { return (T *)p; }
};

constexpr int kStages = 8;
// Tunable launch shapes ("sites"): waves per workgroup of the AEV forward and
// backward kernels, column-tile width of each dense-layer GEMM.
enum { kDescAev = 0, kDescDp = 1 };  // descriptor kinds
enum { kSiteAevFwd = 0, kSiteAevBwd = 1, kSiteGemmFwd = 2, kSiteGemmBwd = 10, kSiteGemmOut = 18,
       kSiteChain = 19, kTuneSites = 20 };
constexpr int kMaxTimedCalls = 4096;  // timed calls held between two reads
const char *kStageNames[kStages] = {"ingest", "cells", "neighbours", "buckets",
                                    "aev_fwd", "mlp", "aev_bwd", "reduce"};

}  // namespace

// Pinned staging of per-call descriptors.  A call copies its descriptors
// from the next slot of the ring; it waits only when that slot's previous
// copy (kStageSlots calls back) has not completed yet.
constexpr int kStageSlots = 32;
constexpr size_t kStageInitBytes = 128 * 1024;  // ~1,400 systems' descriptors
struct StageSlot {
  void *p = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

struct LayerW {
  float *W = nullptr;       // [out][in] float32
  float *Wt = nullptr;      // [in][out] float32
  uint16_t *Wb = nullptr;   // [out][in] bf16
  uint16_t *Wtb = nullptr;  // [in][out] bf16
  float *b = nullptr;
  int n_in = 0, n_out = 0;
};

struct nnp_model {
  int device = 0;
  int S = 0, M = 1, L = 1;
  int precision = NNP_FP32;
  float alpha = 0.1f;
  int kind = 0;                          // kDescAev or kDescDp
  AevConst aev{};                        // descriptor of kind kDescAev
  DpConst dp{};                          // descriptor of kind kDescDp
  int D = 0;                             // descriptor length (the networks' input width)
  float rc_desc = 0.f;                   // neighbour-list cutoff of the descriptor (no skin)
  std::vector<std::vector<int>> widths;  // [S][L+1]
  std::vector<int> ldH;                  // [L-1] max width of hidden layer l
  std::vector<LayerW> layers;            // [(M * S + s) * L + l]
  // per species: [D][M * n1] = members' first-layer W^T side by side (dE/dG)
  std::vector<float *> Wdg;
  std::vector<uint16_t *> Wdg_b;
  std::vector<void *> weight_allocs;
  int cap = 256;                         // neighbour capacity per atom
  int ldG = 0;                           // row stride of the AEV buffer G: the AEV length
                                         // rounded up to 32; columns past it stay zero
  size_t G_zeroed = 0;                   // bytes of G cleared since its last growth
  unsigned long long ws_gen = 0;         // counts workspace reallocations (recorded graphs hold its addresses)

  // workspace
  DevBuf pos, sys_of, atom_cell, atom_slot, cell_count, cell_start, cell_atoms, nbr, nbr_cnt;
  DevBuf block_counts, bucket_off, bucket_cnt, perm, row_of_atom, G, dG, e_atom, W_atom, partial;
  DevBuf desc, status, state, e_mem, dp_rec;  // desc: the per-call descriptors (desc_layout)
  DevBuf Ffix;                           // AEV models: forces in 64-bit fixed point [N][3]
  DevBuf gmask;                          // AEV models: per G row, its possibly non-zero 16-column halves
  DevBuf wave_atom;                      // AEV models: centre of each wave of the per-centre kernels
  size_t max_lds = 64 * 1024;            // LDS bytes one workgroup may use on this device
  std::vector<DevBuf> H, Gd;
  // fused hidden-layer chain (bfloat16 models whose hidden widths allow it)
  bool chain = false;
  bool chain_rt2 = false;                // 64-row workgroups fit the LDS
  DevBuf chain_nets;                     // [member][species] ChainNet
  ChainLaunch chain_proto{};             // strides and LDS layout, filled at creation
  size_t chain_lds = 0;
  // host staging (pinned) for per-call descriptors: a ring of slots, each
  // reused once the copy that last read it has completed
  StageSlot stage[kStageSlots];
  int stage_next = 0;
  // tuned launch shapes (0: default) and the per-site events of a tuning run
  int tune_val[kTuneSites] = {};
  bool tuning = false;
  bool tune_hit[kTuneSites] = {};
  hipEvent_t tune_ev[kTuneSites][2] = {};
  // timing: one set of stage-boundary events per timed call, kept until read
  bool timing = false;
  int timed_stage = -1;  // >= 0: only this stage's two boundary events are recorded
  std::vector<std::array<hipEvent_t, kStages + 1>> evsets;
  int ev_used = 0;       // sets recorded since the last read
  int last_stages = 0;

  LayerW &layer(int m, int s, int l) { return layers[((size_t)m * S + s) * L + l]; }
};

// A persistent pool of neighbour lists: each system of a call owns a range of
// slots (one per atom) for its rows, counts and per-atom state, so its list is
// reused across calls until an atom has moved more than half the skin.
struct nnp_nlist {
  int device = 0;
  int64_t slots = 0;
  int cap = 0;
  float skin = 0.f;
  DevBuf nbr, cnt, state, stats;
  // what each system's rows were last built for, by its first slot: box
  // lengths, list cutoff (model cutoff + skin) and atom count.  A call whose
  // system differs in any of them (another model's cutoff, a changed box, a
  // new system in the slots) rebuilds that system's rows.
  struct Built {
    float L[3];
    float rc_list;
    int n;
  };
  std::unordered_map<int64_t, Built> built;
};

static void round_bf16_host(const float *src, uint16_t *dst, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    uint32_t u;
    memcpy(&u, &src[i], 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    dst[i] = (uint16_t)(u >> 16);
  }
}

static int upload(nnp_model *m, const void *host, size_t bytes, void **dev) {
  HIP_TRY(hipMalloc(dev, bytes));
  m->weight_allocs.push_back(*dev);
  HIP_TRY(hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice));
  return NNP_OK;
}

extern "C" const char *nnp_last_error(void) { return g_err.c_str(); }

extern "C" void nnp_destroy(nnp_model *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (void *p : m->weight_allocs) (void)hipFree(p);
  DevBuf *bufs[] = {&m->pos, &m->sys_of, &m->atom_cell, &m->atom_slot, &m->cell_count,
                    &m->cell_start, &m->cell_atoms, &m->nbr, &m->nbr_cnt, &m->block_counts,
                    &m->bucket_off, &m->bucket_cnt, &m->perm, &m->row_of_atom, &m->G, &m->dG,
                    &m->e_atom, &m->W_atom, &m->partial, &m->desc, &m->status, &m->state, &m->e_mem,
                    &m->chain_nets, &m->dp_rec, &m->Ffix, &m->gmask, &m->wave_atom};
  for (DevBuf *b : bufs) b->release();
  for (auto &b : m->H) b.release();
  for (auto &b : m->Gd) b.release();
  for (StageSlot &ss : m->stage) {
    if (ss.p) (void)hipHostFree(ss.p);
    if (ss.done) (void)hipEventDestroy(ss.done);
  }
  for (auto &set : m->evsets)
    for (auto &e : set)
      if (e) (void)hipEventDestroy(e);
  for (auto &pair : m->tune_ev)
    for (auto &e : pair)
      if (e) (void)hipEventDestroy(e);
  delete m;
}

// Network half of a model description (shared by both descriptor kinds).
struct NetArgs {
  int n_ensemble;
  const int *n_layers;
  const int *widths;
  const float *weights;
  float celu_alpha;
  int precision;
};

static int create_networks(const NetArgs *d, nnp_model *m);

static int create_impl(const nnp_model_desc *dd, nnp_model *m) {
  const nnp_aev_params &a = dd->aev;
  if (a.n_species < 1 || a.n_species > kMaxSpecies)
    return fail(NNP_EUNSUPPORTED, "n_species must be in 1..%d (got %d)", kMaxSpecies, a.n_species);
  if (a.n_shf_rad != kNShfRad || a.n_shf_ang != kNShfAng || a.n_shf_z != kNShfZ)
    return fail(NNP_EUNSUPPORTED, "this build runs 16 radial, 4 angular-radial and 8 angle shifts");
  if (!a.shf_rad || !a.shf_ang || !a.shf_z) return fail(NNP_EINVAL, "null shift array");
  if (!(a.rc_rad > 0.f) || !(a.rc_ang > 0.f) || a.rc_ang > a.rc_rad)
    return fail(NNP_EUNSUPPORTED, "need 0 < rc_ang <= rc_rad");
  if (!(a.zeta >= 1.f)) return fail(NNP_EUNSUPPORTED, "zeta must be >= 1");
  const int S = a.n_species;
  m->S = S;
  AevConst &c = m->aev;
  c.rc_r = a.rc_rad; c.eta_r = a.eta_rad; c.rc_a = a.rc_ang; c.eta_a = a.eta_ang;
  c.zeta = a.zeta; c.scale = a.radial_scale;
  for (int k = 0; k < kNShfRad; ++k) c.shf_r[k] = a.shf_rad[k];
  for (int k = 0; k < kNShfAng; ++k) c.shf_a[k] = a.shf_ang[k];
  for (int k = 0; k < kNShfZ; ++k) {
    c.hcz[k] = (float)(0.5 * std::cos((double)a.shf_z[k]));
    c.hsz[k] = (float)(0.5 * std::sin((double)a.shf_z[k]));
  }
  c.S = S;
  c.rad_len = S * kNShfRad;
  c.D = c.rad_len + S * (S + 1) / 2 * kAngBlock;
  m->kind = kDescAev;
  m->D = c.D;
  m->rc_desc = a.rc_rad;
  const NetArgs net{dd->n_ensemble, dd->n_layers, dd->widths, dd->weights, dd->celu_alpha, dd->precision};
  return create_networks(&net, m);
}

static int create_dp_impl(const nnp_dp_model_desc *dd, nnp_model *m) {
  const nnp_dp_params &p = dd->dp;
  if (p.n_species < 1 || p.n_species > kMaxSpecies)
    return fail(NNP_EUNSUPPORTED, "n_species must be in 1..%d (got %d)", kMaxSpecies, p.n_species);
  if (!p.sel) return fail(NNP_EINVAL, "null sel array");
  if (!(p.rc > 0.f) || !(p.rc < 1e3f)) return fail(NNP_EINVAL, "cutoff must be positive and finite");
  DpConst &c = m->dp;
  memset(&c, 0, sizeof c);
  int slots = 0;
  for (int s = 0; s < p.n_species; ++s) {
    if (p.sel[s] < 0) return fail(NNP_EINVAL, "sel must be >= 0");
    c.sel[s] = p.sel[s];
    c.soff[s] = slots;
    slots += p.sel[s];
    if (slots > kDpMaxSlots) return fail(NNP_EUNSUPPORTED, "at most %d neighbour slots in total", kDpMaxSlots);
  }
  if (slots < 1) return fail(NNP_EINVAL, "sel must keep at least one neighbour");
  c.S = p.n_species;
  c.n_slots = slots;
  c.D = 4 * slots;
  c.ldm = slots + 2;
  c.rc2 = (double)p.rc * (double)p.rc;
  m->S = p.n_species;
  m->kind = kDescDp;
  m->D = c.D;
  // the lists reach 1e-3 A past the cutoff: every neighbour the float64
  // cutoff test admits is in them whatever the float32 rounding
  m->rc_desc = p.rc + 1e-3f;
  const NetArgs net{dd->n_ensemble, dd->n_layers, dd->widths, dd->weights, dd->celu_alpha, dd->precision};
  return create_networks(&net, m);
}

static int create_networks(const NetArgs *d, nnp_model *m) {
  if (d->n_ensemble < 1) return fail(NNP_EINVAL, "n_ensemble must be >= 1");
  if (d->n_ensemble > kMaxMembers) return fail(NNP_EUNSUPPORTED, "at most %d ensemble members", kMaxMembers);
  if (!d->n_layers || !d->widths || !d->weights) return fail(NNP_EINVAL, "null network array");
  if (d->precision != NNP_FP32 && d->precision != NNP_BF16) return fail(NNP_EINVAL, "bad precision");
  if (!(d->celu_alpha > 0.f)) return fail(NNP_EINVAL, "celu_alpha must be > 0");
  const int S = m->S;
  m->M = d->n_ensemble;
  m->precision = d->precision;
  m->alpha = d->celu_alpha;
  const int L = d->n_layers[0];
  if (L < 1) return fail(NNP_EINVAL, "n_layers must be >= 1");
  if (L > 9) return fail(NNP_EUNSUPPORTED, "at most 9 layers per network");
  for (int s = 0; s < S; ++s)
    if (d->n_layers[s] != L)
      return fail(NNP_EUNSUPPORTED, "all species must have the same number of layers");
  m->L = L;
  m->widths.assign(S, std::vector<int>(L + 1));
  for (int s = 0; s < S; ++s)
    for (int l = 0; l <= L; ++l) {
      int w = d->widths[s * (L + 1) + l];
      if (w < 1) return fail(NNP_EINVAL, "width must be >= 1");
      if (l > 0 && l < L && w % 8 != 0)
        return fail(NNP_EUNSUPPORTED, "hidden widths must be multiples of 8");
      m->widths[s][l] = w;
    }
  for (int s = 0; s < S; ++s) {
    if (m->widths[s][0] != m->D) return fail(NNP_EINVAL, "first width must be the descriptor length %d", m->D);
    if (m->widths[s][L] != 1) return fail(NNP_EINVAL, "last width must be 1");
  }
  m->ldG = (m->D + 31) / 32 * 32;
  m->ldH.assign(std::max(L - 1, 0), 0);
  for (int l = 0; l + 1 < L; ++l)
    for (int s = 0; s < S; ++s) m->ldH[l] = std::max(m->ldH[l], m->widths[s][l + 1]);
  m->H.resize(std::max(L - 1, 0));
  m->Gd.resize(std::max(L - 1, 0));

  HIP_TRY(hipGetDevice(&m->device));
  {
    int max_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, m->device));
    m->max_lds = (size_t)max_lds;
  }
  m->layers.resize((size_t)m->M * S * L);
  const float *wp = d->weights;
  std::vector<float> tmp;
  std::vector<uint16_t> tb;
  for (int mb = 0; mb < m->M; ++mb)
    for (int s = 0; s < S; ++s)
      for (int l = 0; l < L; ++l) {
        LayerW &lw = m->layer(mb, s, l);
        lw.n_in = m->widths[s][l];
        lw.n_out = m->widths[s][l + 1];
        size_t nw = (size_t)lw.n_in * lw.n_out;
        int rc;
        if ((rc = upload(m, wp, nw * 4, (void **)&lw.W))) return rc;
        tmp.resize(nw);
        for (int o = 0; o < lw.n_out; ++o)
          for (int k = 0; k < lw.n_in; ++k) tmp[(size_t)k * lw.n_out + o] = wp[(size_t)o * lw.n_in + k];
        if ((rc = upload(m, tmp.data(), nw * 4, (void **)&lw.Wt))) return rc;
        if (m->precision == NNP_BF16) {
          tb.resize(nw);
          if (l == 0) {
            // first layer: rows padded with zeros to the stride of G
            std::vector<uint16_t> pad((size_t)lw.n_out * m->ldG, 0);
            for (int o = 0; o < lw.n_out; ++o)
              round_bf16_host(wp + (size_t)o * lw.n_in, pad.data() + (size_t)o * m->ldG, lw.n_in);
            if ((rc = upload(m, pad.data(), pad.size() * 2, (void **)&lw.Wb))) return rc;
          } else {
            round_bf16_host(wp, tb.data(), nw);
            if ((rc = upload(m, tb.data(), nw * 2, (void **)&lw.Wb))) return rc;
          }
          round_bf16_host(tmp.data(), tb.data(), nw);
          if ((rc = upload(m, tb.data(), nw * 2, (void **)&lw.Wtb))) return rc;
        }
        wp += nw;
        if ((rc = upload(m, wp, (size_t)lw.n_out * 4, (void **)&lw.b))) return rc;
        wp += lw.n_out;
      }
  if (L >= 2) {
    m->Wdg.assign(S, nullptr);
    m->Wdg_b.assign(S, nullptr);
    const float *base = d->weights;
    // offsets of (member, species) first layers in the flat weight array
    std::vector<size_t> off((size_t)m->M * S);
    size_t o = 0;
    for (int mb = 0; mb < m->M; ++mb)
      for (int s = 0; s < S; ++s) {
        off[(size_t)mb * S + s] = o;
        for (int l = 0; l < L; ++l) o += (size_t)m->widths[s][l] * m->widths[s][l + 1] + m->widths[s][l + 1];
      }
    for (int s = 0; s < S; ++s) {
      const int D = m->widths[s][0], n1 = m->widths[s][1], MK = m->M * n1;
      std::vector<float> cat((size_t)D * MK);
      for (int mb = 0; mb < m->M; ++mb) {
        const float *W0 = base + off[(size_t)mb * S + s];  // [n1][D]
        for (int k = 0; k < n1; ++k)
          for (int dd = 0; dd < D; ++dd) cat[(size_t)dd * MK + (size_t)mb * n1 + k] = W0[(size_t)k * D + dd];
      }
      int rc;
      if ((rc = upload(m, cat.data(), cat.size() * 4, (void **)&m->Wdg[s]))) return rc;
      if (m->precision == NNP_BF16) {
        std::vector<uint16_t> cb(cat.size());
        round_bf16_host(cat.data(), cb.data(), cat.size());
        if ((rc = upload(m, cb.data(), cb.size() * 2, (void **)&m->Wdg_b[s]))) return rc;
      }
    }
  }
  // fused chain: bfloat16, 2..4 hidden layers after the first, widths that are
  // multiples of 32 and at most 256, activation tiles within 64 KB of LDS
  if (m->precision == NNP_BF16 && L >= 3 && L - 2 <= kChainMax) {
    bool ok = true;
    size_t lds = 0;
    ChainLaunch &cp = m->chain_proto;
    for (int l = 0; l + 1 < L; ++l) {
      for (int s = 0; s < S; ++s) {
        const int w = m->widths[s][l + 1];
        ok = ok && w % 32 == 0 && w <= 256;
      }
      if (l <= kChainMax) {
        cp.lds_off[l] = (int)lds;
        cp.lds_ld[l] = m->ldH[l] + 8;
        lds += (size_t)kChainRows * (m->ldH[l] + 8) * 2;
      }
    }
    ok = ok && lds <= 64 * 1024;
    if (ok) {
      std::vector<ChainNet> nets((size_t)m->M * S);
      for (int mb = 0; mb < m->M; ++mb)
        for (int s = 0; s < S; ++s) {
          ChainNet &n = nets[(size_t)mb * S + s];
          memset(&n, 0, sizeof n);
          for (int l = 1; l <= L - 2; ++l) {
            LayerW &lw = m->layer(mb, s, l);
            n.W[l - 1] = lw.Wb;
            n.Wt[l - 1] = lw.Wtb;
            n.b[l - 1] = lw.b;
          }
          LayerW &lo = m->layer(mb, s, L - 1);
          n.w_out = lo.W;
          HIP_TRY(hipMemcpy(&n.b_out, lo.b, sizeof(float), hipMemcpyDeviceToHost));
          for (int l = 0; l <= L - 2; ++l) n.width[l] = m->widths[s][l + 1];
        }
      int rc = m->chain_nets.ensure(nets.size() * sizeof(ChainNet));
      if (rc) return rc;
      HIP_TRY(hipMemcpy(m->chain_nets.p, nets.data(), nets.size() * sizeof(ChainNet), hipMemcpyHostToDevice));
      m->chain = true;
      m->chain_lds = lds;
      m->chain_rt2 = 2 * lds <= m->max_lds;
    }
  }
  for (StageSlot &ss : m->stage) {
    HIP_TRY(hipEventCreateWithFlags(&ss.done, hipEventDisableTiming | hipEventDisableSystemFence));
    // coherent: the copy kernel reads it straight from host memory
    HIP_TRY(hipHostMalloc(&ss.p, kStageInitBytes, hipHostMallocCoherent));
    ss.bytes = kStageInitBytes;
  }
  int rc = m->status.ensure(2 * sizeof(int));
  if (rc) return rc;
  HIP_TRY(hipMemset(m->status.p, 0, 2 * sizeof(int)));
  return NNP_OK;
}

static int scratch_init(int dev);

// Runs create on hip_device (< 0: the current device), restoring the
// caller's current device afterwards.
template <class Desc, class Impl>
static int create_on(const Desc *d, int hip_device, nnp_model **out, Impl impl) {
  if (!d || !out) return fail(NNP_EINVAL, "null argument");
  *out = nullptr;
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  if (hip_device >= 0) {
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (hip_device >= n) return fail(NNP_EINVAL, "hip_device %d: the node has %d devices", hip_device, n);
    HIP_TRY(hipSetDevice(hip_device));
  }
  nnp_model *m = new nnp_model();
  int rc = impl(d, m);
  if (rc == NNP_OK) rc = scratch_init(m->device);
  if (rc != NNP_OK) {
    nnp_destroy(m);
  } else {
    *out = m;
  }
  (void)hipSetDevice(prev);
  return rc;
}

extern "C" int nnp_create(const nnp_model_desc *d, int hip_device, nnp_model **out) {
  return create_on(d, hip_device, out, create_impl);
}

extern "C" int nnp_create_dp(const nnp_dp_model_desc *d, int hip_device, nnp_model **out) {
  return create_on(d, hip_device, out, create_dp_impl);
}

extern "C" int nnp_aev_dim(const nnp_model *m) { return m ? m->D : NNP_EINVAL; }

// Layout of the per-call descriptors, the same in pinned staging memory and
// in the device buffer: CallSizes, SysDesc[S], chunk system[n_chunks], chunk first
// atom[n_chunks], first chunk of each system[S + 1], backward centre groups
// int2[n_groups] (8-byte aligned).
struct DescLayout {
  size_t sd, cs, cb, so, gr, total;
  DescLayout(int S, int n_chunks, int n_groups) {
    sd = sizeof(CallSizes);  // the call's sizes come first
    cs = sd + sizeof(SysDesc) * (size_t)S;
    cb = cs + 4 * (size_t)n_chunks;
    so = cb + 4 * (size_t)n_chunks;
    gr = (so + 4 * (size_t)(S + 1) + 7) / 8 * 8;
    total = (gr + 8 * (size_t)n_groups + 15) / 16 * 16;  // moved in 16-byte units
  }
};

// Centres per group of the AEV backward's per-system form.
constexpr int kBwdGroup = 20;
// Groups of a call of small systems: at most this many per atom.
static int64_t max_bwd_groups(int64_t N, int S) { return N / kBwdGroup + S + 1; }

// Buffers for a call of N atoms, S systems, C cells and n_chunks chunks.
// Workspace of a call with N atoms, S systems, C cells and n_chunks
// reduction chunks: f(buffer, bytes) is applied to every buffer (grow it, or
// add up its size).  With pooled lists the neighbour rows, counts and
// per-atom list state live in the pool, not here.
template <class F>
static int for_each_ws(nnp_model *m, int64_t N, int S, int64_t C, int n_chunks, bool pooled, F &&f) {
  const int64_t rows = (N + kTileM - 1) / kTileM * kTileM + (int64_t)m->S * kTileM;
  const int nblk = (int)((N + 1023) / 1024);
  int rc;
#define ENS(buf, bytes) if ((rc = f((buf), (size_t)(bytes)))) return rc
  ENS(m->pos, N * 16);
  ENS(m->sys_of, N * 4);
  ENS(m->atom_cell, N * 4);
  ENS(m->atom_slot, N * 4);
  ENS(m->cell_count, C * 4 + 4);
  ENS(m->cell_start, C * 4 + 8);
  ENS(m->cell_atoms, N * 4);
  if (!pooled) {
    ENS(m->nbr, N * (int64_t)m->cap * 8);
    ENS(m->nbr_cnt, N * 4);
    ENS(m->state, N * (int64_t)sizeof(AtomState));
  }
  ENS(m->block_counts, (int64_t)std::max(nblk, 1) * kMaxSpecies * 4);
  ENS(m->bucket_off, (kMaxSpecies + 1) * 4);
  ENS(m->bucket_cnt, kMaxSpecies * 4);
  ENS(m->perm, rows * 4);
  ENS(m->row_of_atom, N * 4);
  const int esz = m->precision == NNP_BF16 ? 2 : 4;  // activation element size
  ENS(m->G, rows * m->ldG * esz);
  ENS(m->dG, rows * m->D * 4);
  if (m->kind == kDescDp) ENS(m->dp_rec, N * (int64_t)m->dp.ldm * 16);
  ENS(m->e_atom, N * 4);
  if (m->chain) ENS(m->e_mem, rows * m->M * 4);
  ENS(m->W_atom, N * 36);
  ENS(m->partial, (int64_t)n_chunks * 80 + 80);
  ENS(m->desc, DescLayout(S, n_chunks, (int)max_bwd_groups(N, S)).total);
  if (m->kind == kDescAev) ENS(m->Ffix, N * 24);
  if (m->kind == kDescAev) ENS(m->gmask, rows * 8);
  if (m->kind == kDescAev) ENS(m->wave_atom, N * 4);
  for (int l = 0; l + 1 < m->L; ++l) {
    ENS(m->H[l], rows * m->ldH[l] * m->M * esz);
    ENS(m->Gd[l], rows * m->ldH[l] * m->M * esz);
  }
#undef ENS
  return NNP_OK;
}

static int ensure_ws(nnp_model *m, int64_t N, int S, int64_t C, int n_chunks, bool pooled = false) {
  return for_each_ws(m, N, S, C, n_chunks, pooled, [m](DevBuf &b, size_t n) {
    const void *before = b.p;
    const int rc = b.ensure(n);
    if (b.p != before) ++m->ws_gen;
    return rc;
  });
}

// Capacity buckets of graph replay: the smallest of 2^k, 1.25, 1.5 and 1.75
// times 2^k (at least 64) that holds v; a call's launches are sized for its
// bucket (at most 25% above the call).
static int64_t bucket_up(int64_t v) {
  int64_t b = 64;
  while (b < v) b *= 2;
  if (b > 64) {
    const int64_t h = b / 2;
    for (int q = 1; q <= 3; ++q)
      if (h + q * (h / 4) >= v) return h + q * (h / 4);
  }
  return b;
}

// Recorded launch sequences, by everything their launches were recorded
// with: the launch sizes, the call's form and every address a kernel takes.
struct GraphKey {
  int64_t n_launch, s_launch, c_launch, g_launch;
  int all_small, cap;
  const void *ptr[12];
  unsigned long long ws_gen;
  bool operator==(const GraphKey &o) const { return memcmp(this, &o, sizeof o) == 0; }
};
constexpr size_t kMaxGraphs = 48;

namespace nnp {
struct GraphCache {
  struct Entry {
    GraphKey key;
    hipGraphExec_t exec;
    unsigned long long used;
  };
  std::vector<Entry> entries;
  unsigned long long clock = 0;
};
GraphCache *graph_cache_create() { return new GraphCache(); }
int64_t launch_bucket(int64_t v) { return bucket_up(v); }
void graph_cache_destroy(GraphCache *gc) {
  if (!gc) return;
  for (auto &e : gc->entries) (void)hipGraphExecDestroy(e.exec);
  delete gc;
}
}  // namespace nnp

// Fixed device scratch of the allocation-free entry point
// (nnp_energy_forces_noalloc): the whole per-call workspace of one call, on
// every device the library runs on, held until the process ends.  Host code
// uses the address hipGetSymbolAddress returns for the current device (the
// array's name is only a host-side handle), looked up once per device when a
// model is created there.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kScratchDevices];

// Looks up this device's copy of scratch (the device must be current).
static int scratch_init(int dev) {
  if (dev < 0 || dev >= kScratchDevices)
    return fail(NNP_EUNSUPPORTED, "device %d: the fixed scratch covers devices 0..%d", dev, kScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return NNP_OK;
  void *p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch_ptr[dev] = (char *)p;
  return NNP_OK;
}

static char *scratch_base(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// The model's workspace buffers pointed into the fixed scratch for one call;
// the model's own buffers come back when the guard goes out of scope.
struct ScratchViews {
  nnp_model *m = nullptr;
  std::vector<std::pair<DevBuf *, DevBuf>> saved;
  size_t g_zeroed = 0;
  ~ScratchViews() {
    for (auto &sv : saved) *sv.first = sv.second;
    if (m) m->G_zeroed = g_zeroed;
  }
};

static size_t scratch_round(size_t n) { return (n + 255) / 256 * 256; }

// Carves the workspace of a call (N atoms, S systems, C cells, n_chunks
// chunks, lists of the model's own capacity) out of the fixed scratch, or
// refuses the call when it does not fit; nothing is enqueued either way.
static int carve_scratch(nnp_model *m, int64_t N, int S, int64_t C, int n_chunks, ScratchViews &v) {
  char *base = scratch_base(m->device);
  if (!base) return fail(NNP_EDEVICE, "no fixed scratch address for device %d", m->device);
  size_t need = 0;
  for_each_ws(m, N, S, C, n_chunks, false, [&](DevBuf &, size_t n) {
    need += scratch_round(n);
    return 0;
  });
  if (need > kScratchBytes)
    return fail(NNP_EUNSUPPORTED, "the call needs %zu bytes of workspace; the fixed scratch holds %zu", need,
                kScratchBytes);
  v.m = m;
  v.g_zeroed = m->G_zeroed;
  size_t off = 0;
  for_each_ws(m, N, S, C, n_chunks, false, [&](DevBuf &b, size_t n) {
    v.saved.push_back({&b, b});
    b.p = base + off;
    b.bytes = n;
    off += scratch_round(n);
    return 0;
  });
  // whatever an earlier call left there: the AEV rows' padding columns are
  // cleared in this call
  m->G_zeroed = (size_t)-1;
  return NNP_OK;
}

// Cells and reduction chunks reserved for up to max_atoms atoms in
// max_systems systems (non-periodic grids hold at most one cell per atom;
// periodic grids are sized per call).
static int64_t reserve_cells(int64_t max_atoms, int max_systems) { return max_atoms + max_systems; }
static int reserve_chunks(int64_t max_atoms, int max_systems) {
  return (int)(max_atoms / 4096) + max_systems + 1;
}

extern "C" int nnp_reserve(nnp_model *m, int64_t max_atoms, int max_systems, int nbr_capacity) {
  if (!m || max_atoms < 0 || max_systems < 0 || nbr_capacity < 0)
    return fail(NNP_EINVAL, "bad reserve arguments");
  HIP_TRY(hipSetDevice(m->device));
  if (nbr_capacity > 0) {
    if (nbr_capacity > 1024) return fail(NNP_EUNSUPPORTED, "neighbour capacity above 1024");
    int cap = (nbr_capacity + 3) / 4 * 4;
    if (cap != m->cap) {
      m->cap = cap;
      m->nbr.release();
    }
  }
  max_systems = std::max(max_systems, 1);
  return ensure_ws(m, max_atoms, max_systems, reserve_cells(max_atoms, max_systems),
                   reserve_chunks(max_atoms, max_systems));
}

// Hooks for the serving layer (same library).
namespace nnp {

size_t model_workspace_bytes(nnp_model *m, int64_t max_atoms, int max_systems, bool pooled) {
  size_t total = 0;
  max_systems = std::max(max_systems, 1);
  for_each_ws(m, max_atoms, max_systems, reserve_cells(max_atoms, max_systems),
              reserve_chunks(max_atoms, max_systems), pooled, [&](DevBuf &b, size_t n) {
                if (n > b.bytes) total += n + n / 4 + 256;  // what DevBuf::ensure would allocate
                return 0;
              });
  return total;
}

int model_reserve_pooled(nnp_model *m, int64_t max_atoms, int max_systems) {
  HIP_TRY(hipSetDevice(m->device));
  max_systems = std::max(max_systems, 1);
  return ensure_ws(m, max_atoms, max_systems, reserve_cells(max_atoms, max_systems),
                   reserve_chunks(max_atoms, max_systems), true);
}

const int *model_status_word(const nnp_model *m) { return m->status.as<int>(); }
int model_device(const nnp_model *m) { return m->device; }
int model_precision(const nnp_model *m) { return m->precision; }
int model_species(const nnp_model *m) { return m->S; }

}  // namespace nnp

// Appends one event set for a timed call.
static int add_evset(nnp_model *m) {
  std::array<hipEvent_t, kStages + 1> set{};
  // timing only: no system-scope fence at each record (the times are read
  // after the stream has completed)
  for (auto &e : set) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  m->evsets.push_back(set);
  return NNP_OK;
}

// Sets for this many timed calls are created when timing is switched on, so
// that the timed calls themselves create none (event creation can stall the
// host for milliseconds when the runtime grows its signal pool).
constexpr int kTimedSetsAhead = 64;

extern "C" int nnp_set_timing(nnp_model *m, int enable) {
  if (!m) return fail(NNP_EINVAL, "null model");
  if (enable < 0 || enable >= 2 + kStages) return fail(NNP_EINVAL, "timing mode %d: 0, 1 or 2 + a stage index", enable);
  m->timing = enable != 0;
  m->timed_stage = enable >= 2 ? enable - 2 : -1;
  m->ev_used = 0;
  m->last_stages = 0;
  if (m->timing) {
    HIP_TRY(hipSetDevice(m->device));
    while ((int)m->evsets.size() < kTimedSetsAhead) {
      int rc = add_evset(m);
      if (rc) return rc;
    }
  }
  return NNP_OK;
}

// Event set for the next timed call (created on first use past the sets
// made ahead, then reused).
static int next_evset(nnp_model *m, hipEvent_t **out) {
  *out = nullptr;
  if (m->ev_used >= kMaxTimedCalls) return NNP_OK;  // beyond the limit: untimed
  if (m->ev_used == (int)m->evsets.size()) {
    int rc = add_evset(m);
    if (rc) return rc;
  }
  *out = m->evsets[m->ev_used++].data();
  return NNP_OK;
}

extern "C" int nnp_stage_timings(nnp_model *m, float *ms, const char **names, int n) {
  if (!m) return fail(NNP_EINVAL, "null model");
  if (!m->timing || m->last_stages == 0 || m->ev_used == 0) return 0;
  const int k = std::min(n, m->last_stages);
  const int used = m->ev_used;
  const int ts = m->timed_stage;
  if (ts >= m->last_stages) return fail(NNP_EINVAL, "the timed stage is past the calls' stages");
  HIP_TRY(hipEventSynchronize(m->evsets[used - 1][ts >= 0 ? ts + 1 : m->last_stages]));
  for (int q = 0; q < k; ++q) {
    if (names) names[q] = kStageNames[q];
    if (ts >= 0 && q != ts) {  // not recorded
      if (ms) ms[q] = -1.f;
      continue;
    }
    double acc = 0.0;
    for (int c = 0; c < used; ++c) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, m->evsets[c][q], m->evsets[c][q + 1]));
      acc += t;
    }
    if (ms) ms[q] = (float)(acc / used);
  }
  m->ev_used = 0;
  return k;
}

extern "C" int nnp_status(nnp_model *m, void *stream, int *max_nbr) {
  if (!m) return fail(NNP_EINVAL, "null model");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipStreamSynchronize(st));
  int h[2] = {0, 0};
  HIP_TRY(hipMemcpy(h, m->status.p, sizeof h, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(m->status.p, 0, sizeof h));
  if (max_nbr) *max_nbr = h[1];
  if (h[0] & kStatBadSpecies) return fail(NNP_ESPECIES, "an atom's species index is outside the model");
  if (h[0] & kStatBadPairs)
    return fail(NNP_EINVAL, "pair list: an index outside the atoms, a self pair without shift, "
                            "a shift beyond 511 boxes, or a pair listed twice");
  if (h[0] & kStatOverflow)
    return fail(NNP_ECAPACITY, "neighbour list overflow: %d neighbours, capacity %d", h[1], m->cap);
  return NNP_OK;
}

enum Mode { kFull = 0, kAev = 1, kNbr = 2 };

struct CallOut {
  double *energy = nullptr;
  float *forces = nullptr;
  double *virial = nullptr;
  float *atom_energy = nullptr;
  float *aev = nullptr;
  int *nb_counts = nullptr;
  int *nb_entries = nullptr;
  int nb_cap = 0;
  // the workspace comes from the fixed device scratch (nothing is allocated)
  bool no_alloc = false;
};

// Where a call's neighbour lists live: the model's own per-call pool (every
// list rebuilt, no skin) or a persistent nnp_nlist.
struct ListPool {
  nnp_nlist *nl = nullptr;       // null: the model's workspace
  const int64_t *slots = nullptr;  // nl: first slot of each system
  const int32_t *rebuild = nullptr;  // nl: caller-forced rebuilds (nullable)
};

// A caller's pair list (nnp_energy_forces_pairs): one system whose
// neighbour rows come from the list instead of the cell search.
struct PairIn {
  long long n = -1;                 // number of pairs; -1: not the pair-list entry point
  const int32_t *pairs = nullptr;   // DEVICE [n][2]
  const int32_t *shifts = nullptr;  // DEVICE [n][3] lattice shifts, or null (all zero)
  const uint8_t *mask = nullptr;    // DEVICE [N] ML region, or null (every atom)
  int half = 1;                     // 1: each unordered pair once; 0: each direction
};

// Launches the recorded sequence of a call's launches on stream st,
// recording it first (record(cs): the launches, issued on the capture
// stream cs) when no graph was recorded with the same key.  The least
// recently used graph makes room when the cache is full.
template <class Record>
static int replay(nnp_model *m, GraphRun *gr, hipStream_t st, int64_t n_l, int64_t s_l, int64_t c_l,
                  int64_t g_l, bool all_small, int cap, std::initializer_list<const void *> ptrs,
                  Record &&record) {
  GraphCache *gc = gr->cache;
  if (!gc || !gr->capture_stream) return fail(NNP_EINVAL, "graph replay needs a cache and a capture stream");
  GraphKey k;
  memset(&k, 0, sizeof k);
  k.n_launch = n_l;
  k.s_launch = s_l;
  k.c_launch = c_l;
  k.g_launch = g_l;
  k.all_small = all_small ? 1 : 0;
  k.cap = cap;
  int q = 0;
  for (const void *p : ptrs)
    if (q < (int)(sizeof k.ptr / sizeof k.ptr[0])) k.ptr[q++] = p;
  k.ws_gen = m->ws_gen;
  GraphCache::Entry *hit = nullptr;
  for (auto &e : gc->entries)
    if (e.key == k) {
      hit = &e;
      break;
    }
  if (!hit) {
    if (gc->entries.size() >= kMaxGraphs) {
      // the graph leaving may still run on st
      HIP_TRY(hipStreamSynchronize(st));
      auto lru = std::min_element(gc->entries.begin(), gc->entries.end(),
                                  [](const GraphCache::Entry &a, const GraphCache::Entry &b) { return a.used < b.used; });
      (void)hipGraphExecDestroy(lru->exec);
      gc->entries.erase(lru);
    }
    hipStream_t cs = gr->capture_stream;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = record(cs);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    if (rc) {
      if (ec == hipSuccess && g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(NNP_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(NNP_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    gc->entries.push_back({k, ex, 0});
    hit = &gc->entries.back();
    ++gr->captures;
  }
  hit->used = ++gc->clock;
  HIP_TRY(hipGraphLaunch(hit->exec, st));
  ++gr->replays;
  return NNP_OK;
}

static int run(nnp_model *m, int n_sys, const int64_t *offs, const float *coords,
               const int32_t *species, const float *box, const CallOut &o, hipStream_t st, Mode mode,
               const ListPool &lp = ListPool(), const PairIn &pin = PairIn(), GraphRun *gr = nullptr) {
  if (!m) return fail(NNP_EINVAL, "null model");
  if (n_sys < 1) return fail(NNP_EINVAL, "n_systems must be >= 1");
  if (!offs || !box) return fail(NNP_EINVAL, "null host array (batch_offsets / box)");
  if (offs[0] != 0) return fail(NNP_EINVAL, "batch_offsets[0] must be 0");
  for (int s = 0; s < n_sys; ++s)
    if (offs[s + 1] < offs[s]) return fail(NNP_EINVAL, "batch_offsets must be non-decreasing");
  const int64_t N64 = offs[n_sys];
  if (N64 > (int64_t)1 << 28) return fail(NNP_EUNSUPPORTED, "more than 2^28 atoms in one call");
  const int N = (int)N64;
  if (N > 0 && (!coords || !species)) return fail(NNP_EINVAL, "null coords / species");
  if (mode == kFull && !o.energy) return fail(NNP_EINVAL, "null energy");
  if (mode == kFull && o.virial && !o.forces) return fail(NNP_EINVAL, "virial needs forces");
  HIP_TRY(hipSetDevice(m->device));

  nnp_nlist *nl = lp.nl;
  const bool pairs = pin.n >= 0;
  if (pairs) {
    if (n_sys != 1 || nl) return fail(NNP_EINVAL, "a pair list describes one system");
    if (pin.n > 0 && !pin.pairs) return fail(NNP_EINVAL, "null pair list");
  }
  if (nl) {
    if (!lp.slots) return fail(NNP_EINVAL, "null slot offsets");
    if (nl->device != m->device) return fail(NNP_EINVAL, "neighbour-list pool on another device");
    // slot ranges must lie in the pool and must not overlap
    std::vector<std::pair<int64_t, int64_t>> r;
    for (int s = 0; s < n_sys; ++s) {
      const int64_t a = lp.slots[s], n = offs[s + 1] - offs[s];
      if (a < 0 || a + n > nl->slots) return fail(NNP_EINVAL, "system %d: slots outside the pool", s);
      if (n > 0) r.push_back({a, a + n});
    }
    std::sort(r.begin(), r.end());
    for (size_t q = 1; q < r.size(); ++q)
      if (r[q].first < r[q - 1].second) return fail(NNP_EINVAL, "overlapping slot ranges");
  }
  const int cap = nl ? nl->cap : m->cap;
  const float rc_list = m->rc_desc + (nl ? nl->skin : 0.f);
  const float rc_cell = rc_list * (1.0f + 1e-5f);
  std::vector<SysDesc> sd(n_sys);
  std::vector<std::pair<int64_t, nnp_nlist::Built>> built_now;
  auto record_builds = [&]() {
    for (auto &bn : built_now) nl->built[bn.first] = bn.second;
  };
  int64_t C = 0;
  std::vector<int> ch_sys, ch_begin, sys_ch(n_sys + 1);
  for (int s = 0; s < n_sys; ++s) {
    SysDesc &d = sd[s];
    memset(&d, 0, sizeof d);
    const float *b = box + 3 * s;
    bool per = b[0] > 0.f || b[1] > 0.f || b[2] > 0.f;
    if (!(b[0] >= 0.f && b[1] >= 0.f && b[2] >= 0.f) || (per && !(b[0] > 0.f && b[1] > 0.f && b[2] > 0.f)))
      return fail(NNP_EINVAL, "system %d: box must be three positive lengths or all zero", s);
    d.atom_off = (int)offs[s];
    d.n = (int)(offs[s + 1] - offs[s]);
    d.periodic = per ? 1 : 0;
    d.cell_off = (int)C;
    if (pairs) {
      // the caller's shifts refer to its own coordinates: no wrapping, no
      // cells; the box lengths only scale the image vectors
      d.periodic = 0;
      for (int k = 0; k < 3; ++k) d.L[k] = b[k];
      d.state_off = 0;
      d.list_off = 0;
      d.rebuild = 1;
      d.cell_cap = 1;
      C += 1;
      sys_ch[s] = (int)ch_sys.size();
      for (int b0 = d.atom_off; b0 < d.atom_off + d.n; b0 += 4096) {
        ch_sys.push_back(s);
        ch_begin.push_back(b0);
      }
      continue;
    }
    if (nl) {
      d.state_off = lp.slots[s];
      d.list_off = lp.slots[s] * (int64_t)cap;
      d.rebuild = lp.rebuild ? (lp.rebuild[s] != 0) : 0;
      const auto it = nl->built.find(lp.slots[s]);
      const nnp_nlist::Built now = {{b[0], b[1], b[2]}, rc_list, d.n};
      if (it == nl->built.end() || memcmp(&it->second, &now, sizeof now) != 0) {
        d.rebuild = 1;
        built_now.push_back({lp.slots[s], now});  // recorded once the call is enqueued
      }
    } else {
      d.state_off = offs[s];
      d.list_off = offs[s] * (int64_t)cap;
      d.rebuild = 1;
    }
    if (per && (b[0] < 0.25f * rc_list || b[1] < 0.25f * rc_list || b[2] < 0.25f * rc_list))
      return fail(NNP_EUNSUPPORTED, "system %d: periodic box edge below a quarter of the cutoff", s);
    if (per) {
      int64_t cells = 1;
      for (int k = 0; k < 3; ++k) {
        d.L[k] = b[k];
        int nc = std::max(1, (int)std::floor(b[k] / rc_cell));
        nc = std::min(nc, 1024);
        d.nc[k] = nc;
        d.edge[k] = b[k] / nc;
        d.origin[k] = 0.f;
        cells *= nc;
      }
      if (cells > ((int64_t)1 << 26)) return fail(NNP_EUNSUPPORTED, "system %d: too many cells", s);
      d.cell_cap = (int)cells;
    } else {
      // bounding-box grid of cells >= rc; a cell holds ~10-80 atoms at the
      // densities of molecular systems, so a quarter of the atom count bounds it
      d.cell_cap = std::max(1, d.n / 4);
    }
    C += d.cell_cap;
    sys_ch[s] = (int)ch_sys.size();
    for (int b0 = d.atom_off; b0 < d.atom_off + d.n; b0 += 4096) {
      ch_sys.push_back(s);
      ch_begin.push_back(b0);
    }
  }
  sys_ch[n_sys] = (int)ch_sys.size();
  // the AEV kernels' one-wave-per-centre launches take the systems in order
  // of decreasing size, so that the costliest centres do not start last and
  // leave the compute units idle behind them
  {
    std::vector<int> order(n_sys);
    for (int s = 0; s < n_sys; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sd[a].n > sd[b].n; });
    int next = 0;
    for (int s : order) {
      sd[s].order_off = next;
      next += sd[s].n;
    }
  }
  // every system small and without a box: a direct scan per system
  bool all_small = !pairs && N > 0;
  for (int s = 0; s < n_sys && all_small; ++s) all_small = !sd[s].periodic && sd[s].n <= kSmallSystem;
  // and without a persistent list, no system larger than the capacity
  // allows (cap neighbours): the AEV kernels scan each centre's system
  // themselves, and no neighbour list is built
  int max_n = 0;
  for (int s = 0; s < n_sys; ++s) max_n = std::max(max_n, sd[s].n);
  const bool direct = all_small && !nl && m->kind == kDescAev && mode != kNbr && max_n - 1 <= cap;
  // centre groups of the AEV backward's per-system form: consecutive centres
  // of one system, the systems in order of decreasing size (the costliest
  // groups start first)
  std::vector<int2> groups;
  int max_sys_atoms = 0;
  if (all_small && mode == kFull && o.forces && m->kind == kDescAev) {
    std::vector<int> order(n_sys);
    for (int s = 0; s < n_sys; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sd[a].n > sd[b].n; });
    for (int s : order) {
      max_sys_atoms = std::max(max_sys_atoms, sd[s].n);
      for (int p = 0; p < sd[s].n; p += kBwdGroup)
        groups.push_back(make_int2(sd[s].atom_off + p, std::min(kBwdGroup, sd[s].n - p)));
    }
  }
  bool one_chunk_each = true;
  for (int s = 0; s < n_sys && one_chunk_each; ++s) one_chunk_each = sys_ch[s + 1] - sys_ch[s] == 1;
  const int n_chunks = (int)ch_sys.size();
  if (C > ((int64_t)1 << 28)) return fail(NNP_EUNSUPPORTED, "too many cells");
  // Graph replay (a caller's recorded launch sequences, persistent lists,
  // AEV models): every launch is sized for the call's capacity bucket and
  // the kernels read the call's own sizes from its descriptors.  Otherwise
  // the launch sizes are the call's.
  const bool graph = gr && gr->use_graph && m->kind == kDescAev && mode == kFull && nl && !pairs &&
                     !m->timing && !m->tuning && !o.no_alloc && N > 0;
  int N_l = N, S_l = n_sys, chunks_l = n_chunks, groups_l = (int)groups.size();
  int64_t C_l = C;
  if (graph) {
    N_l = (int)bucket_up(N);
    S_l = (int)bucket_up(n_sys);
    // cells: a quarter of the atoms plus one per system bounds the grids of
    // solutes (n/4 cells each) and of boxes at liquid density; sparser boxes
    // take a bucket of their own
    const int64_t c_typ = (int64_t)N_l / 4 + S_l;
    C_l = C <= c_typ ? c_typ : bucket_up(C);
    chunks_l = N_l / 4096 + S_l + 1;
    if (!groups.empty()) {
      groups_l = (int)max_bwd_groups(N_l, S_l);
      max_sys_atoms = kSmallSystem;
    }
    if ((int64_t)N_l > ((int64_t)1 << 28) || C_l > ((int64_t)1 << 28))
      return fail(NNP_EUNSUPPORTED, "too many atoms or cells for a recorded launch");
  }
  ScratchViews views;
  int rc;
  if (o.no_alloc) {
    if (nl || pairs || mode != kFull) return fail(NNP_EINVAL, "the fixed scratch serves plain full calls only");
    // the descriptors must fit the staging slots as they are
    const size_t need = DescLayout(n_sys, n_chunks, (int)groups.size()).total;
    if (need > m->stage[m->stage_next].bytes)
      return fail(NNP_EUNSUPPORTED, "the call's descriptors (%zu bytes) exceed the %zu-byte staging slot", need,
                  m->stage[m->stage_next].bytes);
    rc = carve_scratch(m, N, n_sys, C, n_chunks, views);
  } else {
    rc = ensure_ws(m, N_l, S_l, C_l, chunks_l, nl != nullptr);
  }
  if (rc) return rc;
  if (m->G.bytes != m->G_zeroed) {
    // a newly allocated G: clear it once (with the library's fill kernel) so
    // that the columns past the AEV length (never written) read as zeros in
    // the first-layer GEMM
    launch_fill_i32(m->G.as<int>(), m->G.bytes / 4, 0, st);
    m->G_zeroed = m->G.bytes;
  }

  // stage the per-call descriptors through pinned memory; one copy moves them
  // all into the device buffer of the same layout
  const DescLayout dl(S_l, chunks_l, groups_l);
  const size_t off_sd = dl.sd, off_cs = dl.cs, off_cb = dl.cb, off_so = dl.so, total = dl.total;
  StageSlot &ss = m->stage[m->stage_next];
  m->stage_next = (m->stage_next + 1) % kStageSlots;
  if (ss.pending) {
    // kStageSlots calls are in flight: wait for the oldest one's copy
    HIP_TRY(hipEventSynchronize(ss.done));
    ss.pending = false;
  }
  if (total > ss.bytes) {
    if (ss.p) HIP_TRY(hipHostFree(ss.p));
    ss.p = nullptr;
    ss.bytes = 0;
    size_t nb = (total + total / 2 + 4096 + 15) / 16 * 16;
    HIP_TRY(hipHostMalloc(&ss.p, nb, hipHostMallocCoherent));
    ss.bytes = nb;
  }
  char *hs = (char *)ss.p;
  CallSizes csz;
  memset(&csz, 0, sizeof csz);
  csz.N = N;
  csz.n_sys = n_sys;
  csz.n_cells = (int)C;
  csz.n_chunks = n_chunks;
  csz.n_groups = (int)groups.size();
  memcpy(hs, &csz, sizeof csz);
  memcpy(hs + off_sd, sd.data(), sizeof(SysDesc) * n_sys);
  if (n_chunks) {
    memcpy(hs + off_cs, ch_sys.data(), 4 * (size_t)n_chunks);
    memcpy(hs + off_cb, ch_begin.data(), 4 * (size_t)n_chunks);
  }
  memcpy(hs + off_so, sys_ch.data(), 4 * (size_t)(n_sys + 1));
  if (!groups.empty()) memcpy(hs + dl.gr, groups.data(), 8 * groups.size());
  launch_copy_from_host(hs, m->desc.p, total, st);
  HIP_TRY(hipEventRecord(ss.done, st));
  ss.pending = true;

  // the call's sizes on the device (read by recorded launches)
  const CallSizes *live = (const CallSizes *)m->desc.p;
  const Live lN = graph ? Live(N_l, &live->N) : Live(N);
  const Live lS = graph ? Live(S_l, &live->n_sys) : Live(n_sys);
  const Live lC = graph ? Live((int)C_l, &live->n_cells) : Live((int)C);
  const Live lChunks = graph ? Live(chunks_l, &live->n_chunks) : Live(n_chunks);
  // every launch of the call, on stream st
  auto enqueue = [&](hipStream_t st) -> int {
    int stage = 0;
    hipEvent_t *ev = nullptr;
    if (m->timing && mode == kFull) {
      rc = next_evset(m, &ev);
      if (rc) return rc;
    }
    // stage boundary b: recorded when every stage is timed, or when b opens
    // or closes the one timed stage
    auto mark = [&]() {
      if (ev) {
        const int ts = m->timed_stage;
        if (ts < 0 || stage == ts || stage == ts + 1) (void)hipEventRecord(ev[stage], st);
        ++stage;
      }
    };
    // per-site events while tuning (every site launches at most once per call)
    const bool tuning = m->tuning && mode == kFull;
    auto site_begin = [&](int site) {
      if (tuning) {
        (void)hipEventRecord(m->tune_ev[site][0], st);
        m->tune_hit[site] = true;
      }
    };
    auto site_end = [&](int site) {
      if (tuning) (void)hipEventRecord(m->tune_ev[site][1], st);
    };
    mark();
    SysDesc *dsys = (SysDesc *)(m->desc.as<char>() + off_sd);
    const int *d_chunk_sys = (const int *)(m->desc.as<char>() + off_cs);
    const int *d_chunk_begin = (const int *)(m->desc.as<char>() + off_cb);
    const int *d_sys_chunk_off = (const int *)(m->desc.as<char>() + off_so);
    int *status = m->status.as<int>();
    float4 *pos = m->pos.as<float4>();
    int2 *pool_nbr = nl ? nl->nbr.as<int2>() : m->nbr.as<int2>();
    int *pool_cnt = nl ? nl->cnt.as<int>() : m->nbr_cnt.as<int>();
    AtomState *pool_state = nl ? nl->state.as<AtomState>() : m->state.as<AtomState>();
    if (nl) launch_skin_check(coords, dsys, lS, pool_state, 0.5f * nl->skin, nl->stats.as<int>(), st);
    // AEV models accumulate forces in fixed point (converted by the reduction),
    // DeepPot-style models in float32 straight in the output
    const bool fix_forces = mode == kFull && o.forces && m->kind == kDescAev;
    unsigned long long *Ffix = fix_forces ? m->Ffix.as<unsigned long long>() : nullptr;
    // the launch order of the AEV kernels' centres, for calls of several systems
    int *wave_atom = m->kind == kDescAev && n_sys > 1 && !pairs ? m->wave_atom.as<int>() : nullptr;
    launch_ingest(coords, species, pin.mask, dsys, lS, lN, m->S, pos, m->sys_of.as<int>(), pool_state,
                  status, mode == kFull && !fix_forces ? o.forces : nullptr, Ffix, wave_atom, st);
    mark();
    if (pairs) {
      // the caller's list replaces the cell search (stage "cells" stays empty)
      mark();
      launch_pairs_to_rows(pin.pairs, pin.shifts, pin.n, pin.half, pin.mask, pos, N, sd[0].L, rc_list, cap,
                           pool_nbr, pool_cnt, status, st);
    } else if (all_small) {
      mark();
      if (!direct)
        launch_nbr_small(pos, m->sys_of.as<int>(), dsys, lN, rc_list, cap, pool_nbr, pool_cnt, status, st);
    } else {
      launch_grid(dsys, lS, pos, m->cell_count.as<int>(), rc_list, st);
      launch_cell_count(pos, m->sys_of.as<int>(), dsys, lN, m->cell_count.as<int>(), m->atom_cell.as<int>(),
                        m->atom_slot.as<int>(), st);
      launch_scan(m->cell_count.as<int>(), m->cell_start.as<int>(), lC, st);
      launch_cell_scatter(m->atom_cell.as<int>(), m->atom_slot.as<int>(), m->cell_start.as<int>(), lN,
                          m->cell_atoms.as<int>(), st);
      launch_cell_sort(m->cell_start.as<int>(), lC, m->cell_atoms.as<int>(), st);
      mark();
      launch_nbr_build(pos, m->sys_of.as<int>(), dsys, lS, (int)C_l, m->cell_start.as<int>(),
                       m->cell_atoms.as<int>(), lN, rc_list, cap, pool_nbr, pool_cnt, status, st);
    }
    if (mode == kNbr) {
      launch_export_nbr(pool_nbr, pool_cnt, cap, dsys, m->sys_of.as<int>(), N, o.nb_counts,
                        o.nb_entries, o.nb_cap, st);
      HIP_TRY(hipGetLastError());
      return NNP_OK;
    }
    mark();
    const int nblk = (N_l + 1023) / 1024;
    const int rows = (N_l + kTileM - 1) / kTileM * kTileM + m->S * kTileM;
    launch_species_bucket(pos, wave_atom, lN, m->S, m->block_counts.as<int>(), nblk, m->bucket_off.as<int>(),
                          m->bucket_cnt.as<int>(), m->perm.as<int>(), m->row_of_atom.as<int>(), rows, st);
    // AEV models: the forward records per row the column halves it may have
    // non-zero, and the first layer and the dE/dG product skip what no row
    // of a tile has
    unsigned long long *gmask = m->kind == kDescDp ? nullptr : m->gmask.as<unsigned long long>();
    // atoms outside a caller's mask have no network: zero atomic energy
    // atomic energies go straight to the caller's buffer when one is given
    // (every atom's entry is written each call), else to the workspace
    float *e_atom = o.atom_energy ? o.atom_energy : m->e_atom.as<float>();
    if (pin.mask) launch_fill(e_atom, (size_t)N, 0.f, st);
    mark();
    const int D = m->D;
    const bool bf16 = m->precision == NNP_BF16;
    const bool dp = m->kind == kDescDp;
    const bool want_grad = o.forces != nullptr;
    // descriptor forward into rows of G (the AEV export: float32 rows of the
    // dE/dG buffer, gathered back to atom order)
    auto descriptor = [&](void *Gp, bool g_bf16, int ldg, float4 *rec, unsigned long long *tm, int wpb) {
      if (dp)
        launch_dp_fwd(pos, coords, pool_state, m->sys_of.as<int>(), dsys, pool_nbr, pool_cnt, cap,
                      m->row_of_atom.as<int>(), Gp, g_bf16, ldg, N, m->dp, rec, wpb, st);
      else
        launch_aev_fwd(pos, m->sys_of.as<int>(), dsys, direct ? nullptr : pool_nbr, pool_cnt, cap,
                       m->row_of_atom.as<int>(), Gp, g_bf16, ldg, lN, m->aev, tm, wave_atom,
                       direct ? status : nullptr, wpb, st);
    };
    if (mode == kAev) {
      descriptor(m->dG.p, false, D, nullptr, nullptr, 0);
      launch_gather_rows(m->dG.as<float>(), D, m->row_of_atom.as<int>(), N, D, o.aev, st);
      HIP_TRY(hipGetLastError());
      return NNP_OK;
    }
    site_begin(kSiteAevFwd);
    descriptor(m->G.p, bf16, m->ldG, dp && want_grad ? m->dp_rec.as<float4>() : nullptr, gmask,
               m->tune_val[kSiteAevFwd]);
    site_end(kSiteAevFwd);
    mark();

    // element networks: forward, output layer, backward to dE/dG; every launch
    // covers all species and all ensemble members of one layer index
    const int row_tiles = rows / kTileM;
    const int L = m->L, M = m->M, S = m->S;
    auto common = [&](GemmLaunch &gl) {
      gl.bucket_off = m->bucket_off.as<int>();
      gl.n_groups = S;
      gl.alpha = m->alpha;
      gl.scale = 1.f;
      gl.n_members = M;
      gl.n_seg = 1;
    };
    // with the fused chain only the first layer runs as a separate GEMM
    const bool use_chain = m->chain && bf16;
    for (int l = 0; l + 1 < (use_chain ? 2 : L); ++l) {
      GemmLaunch gl{};
      common(gl);
      gl.A = l == 0 ? m->G.p : m->H[l - 1].p;
      gl.lda = l == 0 ? m->ldG : M * m->ldH[l - 1];
      gl.a_member_stride = l == 0 ? 0 : m->ldH[l - 1];
      gl.C = m->H[l].p;
      gl.ldc = M * m->ldH[l];
      gl.c_member_stride = m->ldH[l];
      if (l == 0) {
        gl.row_mask = gmask;
        gl.bucket_cnt = m->bucket_cnt.as<int>();
      }
      for (int mb = 0; mb < M; ++mb)
        for (int s = 0; s < S; ++s) {
          LayerW &lw = m->layer(mb, s, l);
          GemmGroup &g = gl.g[mb * S + s];
          g.B = bf16 ? (const void *)lw.Wb : (const void *)lw.W;
          g.bias = lw.b;
          g.n_out = lw.n_out;
          g.K = lw.n_in;
          if (l == 0 && bf16) g.K = g.ldb = m->ldG;  // zero-padded columns on both sides
        }
      site_begin(kSiteGemmFwd + l);
      launch_gemm(kEpiFwd, bf16, gl, row_tiles, m->ldH[l], m->tune_val[kSiteGemmFwd + l], st);
      site_end(kSiteGemmFwd + l);
    }
    if (use_chain) {
      ChainLaunch cl = m->chain_proto;
      cl.H0 = (const uint16_t *)m->H[0].p;
      cl.ldh = M * m->ldH[0];
      cl.h_member_stride = m->ldH[0];
      cl.D0 = (uint16_t *)m->Gd[0].p;
      cl.ldd = M * m->ldH[0];
      cl.d_member_stride = m->ldH[0];
      cl.nets = m->chain_nets.as<ChainNet>();
      cl.bucket_off = m->bucket_off.as<int>();
      cl.n_groups = S;
      cl.n_members = M;
      cl.alpha = m->alpha;
      cl.inv_m = 1.0f / (float)M;
      cl.e_mem = m->e_mem.as<float>();
      cl.perm = m->perm.as<int>();
      cl.e_atom = e_atom;
      site_begin(kSiteChain);
      // tuned shape: 4 or 8 waves, plus 10 for 64-row workgroups
      const int tv = m->tune_val[kSiteChain];
      launch_chain(cl, L - 2, want_grad, rows, m->chain_lds, tv % 10 == 4 ? 4 : 8,
                   tv >= 10 && m->chain_rt2 ? 2 : 1, st);
      site_end(kSiteChain);
    } else {
      EnergyLaunch el{};
      el.Hin = L >= 2 ? m->H[L - 2].p : m->G.p;
      el.ldh = L >= 2 ? M * m->ldH[L - 2] : m->ldG;
      el.h_member_stride = L >= 2 ? m->ldH[L - 2] : 0;
      el.Gout = L >= 2 ? m->Gd[L - 2].p : m->dG.p;
      el.ldg = L >= 2 ? M * m->ldH[L - 2] : D;
      el.g_member_stride = L >= 2 ? m->ldH[L - 2] : 0;
      for (int mb = 0; mb < M; ++mb)
        for (int s = 0; s < S; ++s) {
          LayerW &lw = m->layer(mb, s, L - 1);
          el.w[mb * S + s] = lw.W;
          el.b[mb * S + s] = lw.b;
          el.K[s] = lw.n_in;
        }
      el.perm = m->perm.as<int>();
      el.bucket_off = m->bucket_off.as<int>();
      el.n_groups = S;
      el.n_members = M;
      el.e_atom = e_atom;
      el.inv_m = 1.0f / (float)M;
      el.alpha = m->alpha;
      el.hidden = L >= 2;
      el.want_grad = want_grad;
      // the no-hidden-layer form reads float32 AEVs and writes float32 dE/dG
      launch_energy(el, bf16, rows, st);
    }
    if (want_grad) {
      for (int l = L - 2; l >= 1 && !use_chain; --l) {
        GemmLaunch gl{};
        common(gl);
        gl.A = m->Gd[l].p;
        gl.lda = M * m->ldH[l];
        gl.a_member_stride = m->ldH[l];
        gl.C = m->Gd[l - 1].p;
        gl.ldc = M * m->ldH[l - 1];
        gl.c_member_stride = m->ldH[l - 1];
        gl.H = m->H[l - 1].p;
        gl.ldh = M * m->ldH[l - 1];
        gl.h_member_stride = m->ldH[l - 1];
        for (int mb = 0; mb < M; ++mb)
          for (int s = 0; s < S; ++s) {
            LayerW &lw = m->layer(mb, s, l);
            GemmGroup &g = gl.g[mb * S + s];
            g.B = bf16 ? (const void *)lw.Wtb : (const void *)lw.Wt;
            g.n_out = lw.n_in;
            g.K = lw.n_out;
          }
        site_begin(kSiteGemmBwd + l);
        launch_gemm(kEpiBwd, bf16, gl, row_tiles, m->ldH[l - 1], m->tune_val[kSiteGemmBwd + l], st);
        site_end(kSiteGemmBwd + l);
      }
      if (L >= 2) {
        // dE/dG = sum over members of delta_0^m W_0^m: members are K segments
        GemmLaunch gl{};
        common(gl);
        gl.n_members = 1;
        gl.n_seg = M;
        gl.A = m->Gd[0].p;
        gl.lda = M * m->ldH[0];
        gl.a_seg_stride = m->ldH[0];
        gl.C = m->dG.p;
        gl.ldc = D;
        gl.row_mask = gmask;
        gl.bucket_cnt = m->bucket_cnt.as<int>();
        for (int s = 0; s < S; ++s) {
          GemmGroup &g = gl.g[s];
          g.B = bf16 ? (const void *)m->Wdg_b[s] : (const void *)m->Wdg[s];
          g.n_out = D;
          g.K = m->widths[s][1];
        }
        site_begin(kSiteGemmOut);
        launch_gemm(kEpiOut, bf16, gl, row_tiles, D, m->tune_val[kSiteGemmOut], st);
        site_end(kSiteGemmOut);
      }
    }
    mark();
    if (want_grad) {
      site_begin(kSiteAevBwd);
      if (dp) {
        // cells exist for this call unless the pair list or the small-system scan replaced them
        const bool cells = !pairs && !all_small;
        launch_dp_bwd(dsys, n_sys, all_small, cells ? m->cell_start.as<int>() : nullptr,
                      m->cell_atoms.as<int>(), (int)C, m->row_of_atom.as<int>(), m->dG.as<float>(), D, N, m->dp,
                      m->dp_rec.as<float4>(), o.forces, m->W_atom.as<float>(), m->tune_val[kSiteAevBwd], st);
      } else {
        AevBwdGroups gp;
        gp.wave_atom = wave_atom;
        if (!groups.empty()) {
          gp.groups = (const int2 *)(m->desc.as<char>() + dl.gr);
          gp.n_groups = groups_l;
          gp.max_sys_atoms = max_sys_atoms;
          if (graph) gp.live_groups = &live->n_groups;
        } else if (!pairs && !all_small) {
          gp.cell_start = m->cell_start.as<int>();
          gp.cell_atoms = m->cell_atoms.as<int>();
          gp.n_cells = (int)C_l;
          if (graph) gp.live_cells = &live->n_cells;
        }
        launch_aev_bwd(pos, m->sys_of.as<int>(), dsys, direct ? nullptr : pool_nbr, pool_cnt, cap,
                       m->row_of_atom.as<int>(), m->dG.as<float>(), D, lN, m->aev, Ffix,
                       m->W_atom.as<float>(), gp, m->tune_val[kSiteAevBwd], m->max_lds, st);
      }
      site_end(kSiteAevBwd);
    }
    mark();
    launch_reduce(e_atom, want_grad ? m->W_atom.as<float>() : nullptr, dsys, lS,
                  d_chunk_sys, d_chunk_begin, lChunks, d_sys_chunk_off,
                  !graph && one_chunk_each && n_chunks == n_sys,
                  m->partial.as<double>(), o.energy, o.virial, Ffix, o.forces, st);
    mark();
    if (ev) m->last_stages = stage - 1;
    HIP_TRY(hipGetLastError());
    return NNP_OK;
  };
  if (!graph) {
    if (gr && gr->pre) gr->pre(gr->ctx, st, N, n_sys, nullptr);
    int rc2 = enqueue(st);
    if (rc2) return rc2;
    if (gr && gr->post) gr->post(gr->ctx, st, N, n_sys, nullptr);
    HIP_TRY(hipGetLastError());
    if (nl) record_builds();
    return NNP_OK;
  }
  const int rc_replay = replay(m, gr, st, N_l, S_l, C_l, groups_l, all_small, cap,
                {coords, species, o.energy, o.forces, o.virial, o.atom_energy, nl, (const void *)gr->pre,
                 (const void *)gr->post, gr->ctx, m->desc.p, nullptr},
                [&](hipStream_t cs) -> int {
                  if (gr->pre) gr->pre(gr->ctx, cs, N_l, S_l, live);
                  int rc2 = enqueue(cs);
                  if (rc2) return rc2;
                  if (gr->post) gr->post(gr->ctx, cs, N_l, S_l, live);
                  return NNP_OK;
                });
  if (rc_replay == NNP_OK) record_builds();
  return rc_replay;
}

extern "C" int nnp_energy_forces(nnp_model *m, int n_systems, const int64_t *offs, const float *coords,
                                 const int32_t *species, const float *box, double *energy,
                                 float *forces, double *virial, float *atom_energy, void *stream) {
  CallOut o;
  o.energy = energy;
  o.forces = forces;
  o.virial = virial;
  o.atom_energy = atom_energy;
  return run(m, n_systems, offs, coords, species, box, o, (hipStream_t)stream, kFull);
}

extern "C" int nnp_energy_forces_noalloc(nnp_model *m, int n_systems, const int64_t *offs, const float *coords,
                                         const int32_t *species, const float *box, double *energy,
                                         float *forces, double *virial, float *atom_energy, void *stream) {
  CallOut o;
  o.energy = energy;
  o.forces = forces;
  o.virial = virial;
  o.atom_energy = atom_energy;
  o.no_alloc = true;
  return run(m, n_systems, offs, coords, species, box, o, (hipStream_t)stream, kFull);
}

extern "C" int nnp_energy_forces_pairs(nnp_model *m, int64_t n_atoms, const float *coords,
                                       const int32_t *species, const float *box, int64_t n_pairs,
                                       const int32_t *pairs, const int32_t *shifts, int half_list,
                                       const uint8_t *ml_mask, double *energy, float *forces,
                                       double *virial, float *atom_energy, void *stream) {
  if (n_atoms < 0) return fail(NNP_EINVAL, "n_atoms must be >= 0");
  if (n_pairs < 0) return fail(NNP_EINVAL, "n_pairs must be >= 0");
  if (n_pairs > ((int64_t)1 << 40)) return fail(NNP_EUNSUPPORTED, "more than 2^40 pairs");
  if (half_list != 0 && half_list != 1) return fail(NNP_EINVAL, "half_list must be 0 or 1");
  const int64_t offs[2] = {0, n_atoms};
  CallOut o;
  o.energy = energy;
  o.forces = forces;
  o.virial = virial;
  o.atom_energy = atom_energy;
  PairIn pin;
  pin.n = n_pairs;
  pin.pairs = pairs;
  pin.shifts = shifts;
  pin.mask = ml_mask;
  pin.half = half_list;
  return run(m, 1, offs, coords, species, box, o, (hipStream_t)stream, kFull, ListPool(), pin);
}

extern "C" int nnp_debug_aev(nnp_model *m, int n_systems, const int64_t *offs, const float *coords,
                             const int32_t *species, const float *box, float *aev_out, void *stream) {
  if (!aev_out) return fail(NNP_EINVAL, "null aev_out");
  CallOut o;
  o.aev = aev_out;
  return run(m, n_systems, offs, coords, species, box, o, (hipStream_t)stream, kAev);
}

extern "C" int nnp_debug_neighbors(nnp_model *m, int n_systems, const int64_t *offs,
                                   const float *coords, const int32_t *species, const float *box,
                                   int32_t *counts, int32_t *entries, int capacity, void *stream) {
  if (!counts || !entries || capacity < 1) return fail(NNP_EINVAL, "null neighbour outputs");
  CallOut o;
  o.nb_counts = counts;
  o.nb_entries = entries;
  o.nb_cap = capacity;
  return run(m, n_systems, offs, coords, species, box, o, (hipStream_t)stream, kNbr);
}

extern "C" int nnp_autotune(nnp_model *m, int n_systems, const int64_t *offs, const float *coords,
                            const int32_t *species, const float *box, void *stream) {
  if (!m) return fail(NNP_EINVAL, "null model");
  if (n_systems < 1 || !offs) return fail(NNP_EINVAL, "bad batch");
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = offs[n_systems];
  if (N < 1) return fail(NNP_EINVAL, "empty batch");
  for (auto &pair : m->tune_ev)
    for (auto &e : pair)
      if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  double *energy = nullptr;
  float *forces = nullptr;
  if (hipMalloc(&energy, sizeof(double) * n_systems) != hipSuccess ||
      hipMalloc(&forces, sizeof(float) * 3 * (size_t)N) != hipSuccess) {
    (void)hipGetLastError();
    if (energy) (void)hipFree(energy);
    return fail(NNP_ENOMEM, "tuning outputs");
  }
  CallOut o;
  o.energy = energy;
  o.forces = forces;
  // candidates: round r sets every GEMM site to kTn[r], the AEV forward to
  // kWpb[r] waves per workgroup, the AEV backward to kBwd[r] (1: a wave per
  // centre with device atomics; 5, 4, 8: a grouped form with that many
  // waves) and the fused chain to kChainW[r] waves per workgroup
  constexpr int kRounds = 4, kReps = 5;
  const int kTn[kRounds] = {64, 128, 256, 128}, kWpb[kRounds] = {1, 2, 4, 2};
  const int kBwd[kRounds] = {1, 5, 4, 8};
  // chain: 8 or 4 waves on 32 rows, 8 waves on 64 rows (+10) when the LDS allows
  const int kChainW[kRounds] = {8, 4, m->chain_rt2 ? 18 : 8, 8};
  // Every candidate runs once untimed, then the rounds take turns kReps
  // times (so that clock and cache warm-up do not favour a late round), and
  // each candidate keeps its fastest time.
  double t[kTuneSites][kRounds];
  for (auto &row : t)
    for (double &x : row) x = 1e30;
  bool hit[kTuneSites] = {};
  int rc = NNP_OK;
  for (int k = -1; k < kReps && rc == NNP_OK; ++k) {
    for (int r = 0; r < kRounds && rc == NNP_OK; ++r) {
      for (int q = 0; q < kTuneSites; ++q)
        m->tune_val[q] = q == kSiteAevBwd ? kBwd[r] : q < kSiteGemmFwd ? kWpb[r] : q == kSiteChain ? kChainW[r] : kTn[r];
      if (k < 0) {  // warm-up
        rc = run(m, n_systems, offs, coords, species, box, o, st, kFull);
        continue;
      }
      m->tuning = true;
      for (bool &h : m->tune_hit) h = false;
      rc = run(m, n_systems, offs, coords, species, box, o, st, kFull);
      m->tuning = false;
      if (rc) break;
      if (hipStreamSynchronize(st) != hipSuccess) { rc = fail(NNP_EDEVICE, "tuning run failed"); break; }
      for (int q = 0; q < kTuneSites; ++q)
        if (m->tune_hit[q]) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, m->tune_ev[q][0], m->tune_ev[q][1]) == hipSuccess) t[q][r] = std::min(t[q][r], (double)ms);
          hit[q] = true;
        }
    }
  }
  // the fastest candidate of each site that ran (a value tried in two rounds
  // keeps the faster of them)
  for (int q = 0; q < kTuneSites; ++q) {
    m->tune_val[q] = 0;
    if (!hit[q] || rc) continue;
    if (q == kSiteChain) {
      int best = 0;
      for (int r = 1; r < kRounds; ++r) if (t[q][r] < t[q][best]) best = r;
      m->tune_val[q] = kChainW[best];
    } else {
      int best = 0;
      for (int r = 1; r < kRounds; ++r) if (t[q][r] < t[q][best]) best = r;
      m->tune_val[q] = q == kSiteAevBwd ? kBwd[best] : q < kSiteGemmFwd ? kWpb[best] : kTn[best];
    }
  }
  (void)hipFree(energy);
  (void)hipFree(forces);
  return rc;
}

extern "C" int nnp_tuning(const nnp_model *m, int *values, int n) {
  if (!m) return fail(NNP_EINVAL, "null model");
  for (int q = 0; q < std::min(n, (int)kTuneSites); ++q) values[q] = m->tune_val[q];
  return kTuneSites;
}

extern "C" int nnp_nlist_create(nnp_model *m, int64_t slots, int capacity, float skin, nnp_nlist **out) {
  if (!m || !out) return fail(NNP_EINVAL, "null argument");
  *out = nullptr;
  if (slots < 1 || capacity < 1 || !(skin >= 0.f)) return fail(NNP_EINVAL, "bad pool size, capacity or skin");
  if (capacity > 1024) return fail(NNP_EUNSUPPORTED, "neighbour capacity above 1024");
  HIP_TRY(hipSetDevice(m->device));
  nnp_nlist *nl = new nnp_nlist();
  nl->device = m->device;
  nl->slots = slots;
  nl->cap = (capacity + 3) / 4 * 4;
  nl->skin = skin;
  int rc;
  if ((rc = nl->nbr.ensure((size_t)slots * nl->cap * 8)) || (rc = nl->cnt.ensure((size_t)slots * 4)) ||
      (rc = nl->state.ensure((size_t)slots * sizeof(AtomState))) || (rc = nl->stats.ensure(16))) {
    nnp_nlist_destroy(nl);
    return rc;
  }
  hipError_t e = hipMemset(nl->stats.p, 0, 16);
  if (e != hipSuccess) {
    nnp_nlist_destroy(nl);
    return fail(NNP_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
  }
  *out = nl;
  return NNP_OK;
}

extern "C" void nnp_nlist_destroy(nnp_nlist *nl) {
  if (!nl) return;
  (void)hipSetDevice(nl->device);
  (void)hipDeviceSynchronize();
  nl->nbr.release();
  nl->cnt.release();
  nl->state.release();
  nl->stats.release();
  delete nl;
}

extern "C" int nnp_nlist_builds(nnp_nlist *nl, void *stream, int64_t *builds) {
  if (!nl || !builds) return fail(NNP_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(nl->device));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int h = 0;
  HIP_TRY(hipMemcpy(&h, nl->stats.p, sizeof h, hipMemcpyDeviceToHost));
  *builds = h;
  return NNP_OK;
}

namespace nnp {
int run_nlist(nnp_model *m, nnp_nlist *nl, int n_systems, const int64_t *offs, const int64_t *slots,
              const int32_t *rebuild, const float *coords, const int32_t *species, const float *box,
              double *energy, float *forces, double *virial, float *atom_energy, hipStream_t st,
              GraphRun *gr) {
  if (!nl) return fail(NNP_EINVAL, "null neighbour-list pool");
  CallOut o;
  o.energy = energy;
  o.forces = forces;
  o.virial = virial;
  o.atom_energy = atom_energy;
  ListPool lp;
  lp.nl = nl;
  lp.slots = slots;
  lp.rebuild = rebuild;
  return run(m, n_systems, offs, coords, species, box, o, st, kFull, lp, PairIn(), gr);
}
}  // namespace nnp

extern "C" int nnp_energy_forces_nlist(nnp_model *m, nnp_nlist *nl, int n_systems, const int64_t *offs,
                                       const int64_t *slots, const int32_t *rebuild, const float *coords,
                                       const int32_t *species, const float *box, double *energy,
                                       float *forces, double *virial, float *atom_energy, void *stream) {
  if (!nl) return fail(NNP_EINVAL, "null neighbour-list pool");
  CallOut o;
  o.energy = energy;
  o.forces = forces;
  o.virial = virial;
  o.atom_energy = atom_energy;
  ListPool lp;
  lp.nl = nl;
  lp.slots = slots;
  lp.rebuild = rebuild;
  return run(m, n_systems, offs, coords, species, box, o, (hipStream_t)stream, kFull, lp);
}

namespace nnp {
const int *nlist_counts(const nnp_nlist *nl) { return nl->cnt.as<int>(); }
}  // namespace nnp
