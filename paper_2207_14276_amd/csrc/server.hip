// Continuous-batching server of energy/force requests on one GPU, and the
// host-only scheduler entry points.
//
// Every admitted request keeps its coordinates and species in a device store
// (one slot per atom, the same slots as its persistent neighbour list in the
// pool) for its whole life.  One iteration evaluates the next step of every
// request in flight with a single batched call on the persistent lists
// (rebuilt when an atom has moved more than half the skin), then moves each
// continuing request's atoms with the built-in client: a random walk of
// N(0, sigma^2) per coordinate, drawn on the device from a counter-based
// generator keyed by the request's seed, so a request's trajectory does not
// depend on what it is batched with.  Requests that arrive meanwhile are
// admitted first-come first-served as slots, the per-iteration atom budget
// and the request limit allow; the budget follows from the device memory
// granted to the server.  Iterations are pipelined two deep on the stream:
// the host prepares and enqueues one while the previous runs, and collects
// results (energies of every step, coordinates and forces of the last) when
// an iteration's event has completed.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <unordered_map>
#include <vector>

#include "../../include/nnp.h"
#include "internal.h"
#include "scheduler.h"

using namespace nnp;

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(NNP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

namespace {

// ------------------------------------------------------------------ device

// One request in an iteration, as the gather and walk kernels see it.
struct ServeSys {
  long long slot;   // first store slot
  int off;          // first atom in the batch
  int n;            // atoms
  unsigned key0, key1;  // generator key (the request's seed)
  int step;         // step evaluated in this iteration
  int move;         // nonzero: the request continues; draw its next move
  float sigma;
  int pad;
};

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64-bit multiplies
// with the Weyl-sequence key schedule.
__device__ inline uint4 philox4x32_10(uint4 c, uint2 k) {
  for (int r = 0; r < 10; ++r) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// Index of the system holding batch atom i (systems sorted by offset).
__device__ inline int find_sys(const ServeSys *sys, int n_sys, int i) {
  int lo = 0, hi = n_sys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].off <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Batch coordinates and species from the store.
__global__ void k_gather(const ServeSys *__restrict__ sys, Live n_sys, const float *__restrict__ sx,
                         const int *__restrict__ ss, float *__restrict__ bx, int *__restrict__ bs,
                         Live N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N.get()) return;
  const ServeSys d = sys[find_sys(sys, n_sys.get(), i)];
  const long long g = d.slot + (i - d.off);
  bx[3 * (size_t)i] = sx[3 * g];
  bx[3 * (size_t)i + 1] = sx[3 * g + 1];
  bx[3 * (size_t)i + 2] = sx[3 * g + 2];
  bs[i] = ss[g];
}

// The client's move after step `step`: x += sigma * z with z ~ N(0, 1) from
// Philox (counter = (local atom, step + 1, 0, 0), key = seed) and the
// Box-Muller transform (three of its four normals are used).
__global__ void k_walk(const ServeSys *__restrict__ sys, Live n_sys, float *__restrict__ sx, Live N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N.get()) return;
  const ServeSys d = sys[find_sys(sys, n_sys.get(), i)];
  if (!d.move) return;
  const int a = i - d.off;
  const uint4 r = philox4x32_10(make_uint4((unsigned)a, (unsigned)(d.step + 1), 0u, 0u),
                                make_uint2(d.key0, d.key1));
  const float k32 = 2.3283064365386963e-10f;  // 2^-32
  const float u1 = ((float)r.x + 1.0f) * k32;  // (0, 1]
  const float u2 = (float)r.y * k32;           // [0, 1)
  const float u3 = ((float)r.z + 1.0f) * k32;
  const float u4 = (float)r.w * k32;
  const float twopi = 6.283185307179586f;
  const float m1 = sqrtf(-2.0f * logf(fminf(u1, 1.0f)));
  const float m2 = sqrtf(-2.0f * logf(fminf(u3, 1.0f)));
  const long long g = d.slot + a;
  sx[3 * g] += d.sigma * m1 * cosf(twopi * u2);
  sx[3 * g + 1] += d.sigma * m1 * sinf(twopi * u2);
  sx[3 * g + 2] += d.sigma * m2 * cosf(twopi * u4);
}

// Largest neighbour count of each request's atoms in the list pool (counts
// are kept past the capacity, so an overflowing list shows here), one
// workgroup per request.
__global__ void __launch_bounds__(256) k_req_max_count(const ServeSys *__restrict__ sys,
                                                       const int *__restrict__ counts, int *__restrict__ out,
                                                       Live n_sys) {
  __shared__ int red[256 / 64];
  if ((int)blockIdx.x >= n_sys.get()) return;  // the whole workgroup
  const ServeSys d = sys[blockIdx.x];
  int mx = 0;
  for (int a = threadIdx.x; a < d.n; a += blockDim.x) mx = max(mx, counts[d.slot + a]);
  for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = mx;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// Clears the model's device flags before an iteration (a kernel, not a
// memset: the iteration stays free of memset nodes).
__global__ void k_clear_flags(int *status) {
  if (threadIdx.x < 2) status[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ host

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Pinned {
  void *p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return NNP_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    size_t nb = need + need / 2 + 4096;
    if (hipHostMalloc(&p, nb, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(NNP_ENOMEM, "pinned host allocation of %zu bytes failed", nb);
    }
    bytes = nb;
    return NNP_OK;
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

struct DevMem {
  void *p = nullptr;
  int alloc(size_t bytes) {
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(NNP_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    return NNP_OK;
  }
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  template <class T> T *as() const { return (T *)p; }
};

// A submitted request: its inputs until admission, its results after.
struct Request {
  int n = 0;
  int n_steps = 0;
  float box[3] = {0.f, 0.f, 0.f};
  float sigma = 0.f;
  uint64_t seed = 0;
  std::vector<float> coords;     // start coordinates (freed once uploaded)
  std::vector<int32_t> species;  // (freed once uploaded)
  std::vector<double> energy;    // per step
  std::vector<float> last_coords, last_forces;
  int error = NNP_OK;            // NNP_ECAPACITY: stopped, its list overflowed
  int max_count = 0;             // the neighbour count that overflowed
};

// Host side of one launched iteration (a ring of these backs the pipeline).
struct Iteration {
  Pinned up;    // uploads of admitted requests, then the ServeSys table
  Pinned out;   // status word, energies [S], largest neighbour counts [S], then coords and
                // forces [N][3] if wanted
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<LaunchItem> items;
  std::vector<int64_t> offs;
  bool want_xf = false;
  size_t off_energy = 0, off_cnt = 0, off_x = 0, off_f = 0;
};

constexpr int kDepth = 2;   // iterations in flight
constexpr int kRing = kDepth + 1;

}  // namespace

struct nnp_server {
  nnp_model *model = nullptr;
  nnp_nlist *list = nullptr;
  int device = 0;
  int64_t slots = 0;
  int64_t max_batch = 0;
  int max_active = 0;
  int cap = 0;
  float skin = 0.f;
  uint64_t granted = 0;
  double t0 = 0.0;
  std::unique_ptr<Scheduler> sched;
  DevMem store_x, store_s;          // [slots][3] f32, [slots] i32
  DevMem bx, bs, bf, be, bsys;      // batch coords, species, forces, energies, ServeSys table
  DevMem bcnt;                      // largest neighbour count per request [max_active]
  std::unordered_map<int64_t, Request> reqs;
  Iteration ring[kRing];
  std::deque<int> inflight;         // ring indices, oldest first
  int next_ring = 0;
  int64_t next_id = 0;
  int n_species = 0;
  int sticky = NNP_OK;              // an unexpected device flag (species checked at submission)
  int64_t max_batch_seen = 0;
  std::vector<int64_t> ready;       // finished, not yet handed out
  // iterations as recorded graphs: the cache, the recording stream, counters
  GraphRun gr;
  hipStream_t cap_stream = nullptr;
  double host_s = 0.0;              // host time in launch_iteration
};

namespace {

double server_clock(const nnp_server *s) { return now_s() - s->t0; }

// Waits for the oldest iteration in flight and files its results.
int retire_one(nnp_server *s, bool block) {
  if (s->inflight.empty()) return NNP_OK;
  Iteration &it = s->ring[s->inflight.front()];
  if (block) {
    HIP_TRY(hipEventSynchronize(it.done));
  } else {
    hipError_t q = hipEventQuery(it.done);
    if (q == hipErrorNotReady) return 1;
    if (q != hipSuccess) return fail(NNP_EDEVICE, "hipEventQuery: %s", hipGetErrorString(q));
  }
  const double t = server_clock(s);
  const char *o = (const char *)it.out.p;
  const int status = *(const int *)o;
  // a neighbour overflow is a request's own failure (below); anything else
  // should not happen (species are checked at submission)
  if ((status & ~kStatOverflow) && s->sticky == NNP_OK) s->sticky = NNP_ESPECIES;
  const double *E = (const double *)(o + it.off_energy);
  const int *cnt = (const int *)(o + it.off_cnt);
  const float *X = (const float *)(o + it.off_x);
  const float *F = (const float *)(o + it.off_f);
  for (size_t q = 0; q < it.items.size(); ++q) {
    const LaunchItem &li = it.items[q];
    Request &r = s->reqs[li.id];
    if (r.error) continue;  // stopped in an earlier iteration: this step's results are void
    if (cnt[q] > s->cap) {
      // this request's list overflowed: it stops alone, the others go on
      r.error = NNP_ECAPACITY;
      r.max_count = cnt[q];
      if (s->sched->fail(li.id, t)) s->ready.push_back(li.id);
      continue;
    }
    r.energy[li.step] = E[q];
    if (li.last) {
      const size_t a = (size_t)it.offs[q] * 3, n3 = (size_t)li.n_atoms * 3;
      r.last_coords.assign(X + a, X + a + n3);
      r.last_forces.assign(F + a, F + a + n3);
    }
    if (s->sched->complete(li.id, t)) s->ready.push_back(li.id);
  }
  it.busy = false;
  it.items.clear();
  s->inflight.pop_front();
  return NNP_OK;
}

int retire_ready(nnp_server *s) {
  while (!s->inflight.empty()) {
    int rc = retire_one(s, false);
    if (rc == 1) return NNP_OK;
    if (rc) return rc;
  }
  return NNP_OK;
}

// The server's launches before and after the evaluation of an iteration,
// sized for n_l atoms and s_l requests; live (when recorded): the device
// address of the iteration's own sizes.
void serve_pre(void *ctx, hipStream_t st, int n_l, int s_l, const CallSizes *live) {
  nnp_server *s = (nnp_server *)ctx;
  const Live N(n_l, live ? &live->N : nullptr), S(s_l, live ? &live->n_sys : nullptr);
  k_clear_flags<<<1, 64, 0, st>>>(const_cast<int *>(model_status_word(s->model)));
  k_gather<<<(unsigned)((n_l + 255) / 256), 256, 0, st>>>(s->bsys.as<ServeSys>(), S, s->store_x.as<float>(),
                                                          s->store_s.as<int>(), s->bx.as<float>(),
                                                          s->bs.as<int>(), N);
}

void serve_post(void *ctx, hipStream_t st, int n_l, int s_l, const CallSizes *live) {
  nnp_server *s = (nnp_server *)ctx;
  const Live N(n_l, live ? &live->N : nullptr), S(s_l, live ? &live->n_sys : nullptr);
  k_req_max_count<<<(unsigned)s_l, 256, 0, st>>>(s->bsys.as<ServeSys>(), nlist_counts(s->list),
                                                 s->bcnt.as<int>(), S);
  k_walk<<<(unsigned)((n_l + 255) / 256), 256, 0, st>>>(s->bsys.as<ServeSys>(), S, s->store_x.as<float>(), N);
}

int launch_iteration_impl(nnp_server *s, hipStream_t st, bool *launched);

// Admits what fits and launches one iteration if any request is in flight
// (host time counted).
int launch_iteration(nnp_server *s, hipStream_t st, bool *launched) {
  const double t0 = now_s();
  const int rc = launch_iteration_impl(s, st, launched);
  s->host_s += now_s() - t0;
  return rc;
}

int launch_iteration_impl(nnp_server *s, hipStream_t st, bool *launched) {
  *launched = false;
  const double t = server_clock(s);
  std::vector<int64_t> admitted = s->sched->admit(t);
  std::vector<LaunchItem> items = s->sched->launch();
  if (items.empty()) return NNP_OK;
  const int k = s->next_ring;
  Iteration &it = s->ring[k];
  if (it.busy) return fail(NNP_EDEVICE, "iteration ring overrun");
  const int S = (int)items.size();

  // uploads and the per-request table through pinned memory
  size_t up_bytes = 0;
  for (int64_t id : admitted) up_bytes += (size_t)s->reqs[id].n * 16;
  const size_t off_sys = (up_bytes + 255) / 256 * 256;
  int rc = it.up.ensure(off_sys + sizeof(ServeSys) * (size_t)S);
  if (rc) return rc;
  char *up = (char *)it.up.p;
  size_t pos = 0;
  for (int64_t id : admitted) {
    Request &r = s->reqs[id];
    const Job *j = s->sched->job(id);
    const size_t nx = (size_t)r.n * 12, ns = (size_t)r.n * 4;
    memcpy(up + pos, r.coords.data(), nx);
    memcpy(up + pos + nx, r.species.data(), ns);
    HIP_TRY(hipMemcpyAsync(s->store_x.as<float>() + 3 * j->slot, up + pos, nx, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->store_s.as<int>() + j->slot, up + pos + nx, ns, hipMemcpyHostToDevice, st));
    pos += nx + ns;
    std::vector<float>().swap(r.coords);
    std::vector<int32_t>().swap(r.species);
  }
  ServeSys *tab = (ServeSys *)(up + off_sys);
  it.offs.assign(S + 1, 0);
  std::vector<int64_t> slots(S);
  std::vector<int32_t> rebuild(S);
  std::vector<float> boxes(3 * (size_t)S);
  bool want_xf = false;
  for (int q = 0; q < S; ++q) {
    const LaunchItem &li = items[q];
    const Request &r = s->reqs[li.id];
    ServeSys &d = tab[q];
    d.slot = li.slot;
    d.off = (int)it.offs[q];
    d.n = li.n_atoms;
    d.key0 = (unsigned)(r.seed & 0xffffffffu);
    d.key1 = (unsigned)(r.seed >> 32);
    d.step = li.step;
    d.move = li.last ? 0 : 1;
    d.sigma = r.sigma;
    d.pad = 0;
    it.offs[q + 1] = it.offs[q] + li.n_atoms;
    slots[q] = li.slot;
    rebuild[q] = li.step == 0 ? 1 : 0;
    memcpy(&boxes[3 * (size_t)q], r.box, 12);
    want_xf = want_xf || li.last;
  }
  const int64_t N = it.offs[S];
  s->max_batch_seen = std::max(s->max_batch_seen, N);
  HIP_TRY(hipMemcpyAsync(s->bsys.p, tab, sizeof(ServeSys) * (size_t)S, hipMemcpyHostToDevice, st));
  // the evaluation with the server's kernels before (flags, gather) and
  // after (overflow counts, the client's move), as one recorded graph per
  // capacity bucket or launched directly
  rc = run_nlist(s->model, s->list, S, it.offs.data(), slots.data(), rebuild.data(), s->bx.as<float>(),
                 s->bs.as<int32_t>(), boxes.data(), s->be.as<double>(), s->bf.as<float>(), nullptr, nullptr, st,
                 &s->gr);
  if (rc) return rc;

  // results back to the host
  it.off_energy = 16;
  it.off_cnt = it.off_energy + 8 * (size_t)S;
  it.off_x = (it.off_cnt + 4 * (size_t)S + 255) / 256 * 256;
  it.off_f = it.off_x + 12 * (size_t)N;
  rc = it.out.ensure(want_xf ? it.off_f + 12 * (size_t)N : it.off_x);
  if (rc) return rc;
  char *o = (char *)it.out.p;
  HIP_TRY(hipMemcpyAsync(o, model_status_word(s->model), sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(o + it.off_energy, s->be.p, 8 * (size_t)S, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(o + it.off_cnt, s->bcnt.p, 4 * (size_t)S, hipMemcpyDeviceToHost, st));
  if (want_xf) {
    HIP_TRY(hipMemcpyAsync(o + it.off_x, s->bx.p, 12 * (size_t)N, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(o + it.off_f, s->bf.p, 12 * (size_t)N, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipEventRecord(it.done, st));
  it.items.swap(items);
  it.want_xf = want_xf;
  it.busy = true;
  s->inflight.push_back(k);
  s->next_ring = (k + 1) % kRing;
  *launched = true;
  return NNP_OK;
}

}  // namespace

extern "C" int nnp_server_create(nnp_model *m, const nnp_server_opts *o, nnp_server **out) {
  if (!m || !o || !out) return fail(NNP_EINVAL, "null argument");
  *out = nullptr;
  if (o->slots < 1 || o->nbr_capacity < 1 || !(o->skin >= 0.f) || o->max_active < 1 ||
      o->max_batch_atoms < 0)
    return fail(NNP_EINVAL, "bad server options");
  if (o->nbr_capacity > 1024) return fail(NNP_EUNSUPPORTED, "neighbour capacity above 1024");
  const int dev = model_device(m);
  HIP_TRY(hipSetDevice(dev));
  // the server watches the model's device flags: they must start clear
  int rc0 = nnp_status(m, nullptr, nullptr);
  if (rc0) return rc0;
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  const uint64_t budget = o->hbm_budget ? o->hbm_budget : (uint64_t)(0.9 * (double)free_b);
  const int cap = (o->nbr_capacity + 3) / 4 * 4;
  // memory that scales with the slots: store, then the list pool
  const uint64_t per_slot = 16 + (uint64_t)cap * 8 + 4 + sizeof(AtomState);
  const uint64_t fixed = per_slot * (uint64_t)o->slots + 16 + (uint64_t)o->max_active * (sizeof(ServeSys) + 8) + 4096;
  if (fixed > budget)
    return fail(NNP_ENOMEM, "%lld slots need %llu bytes; the budget is %llu", (long long)o->slots,
                (unsigned long long)fixed, (unsigned long long)budget);
  // the largest per-iteration atom count whose batch buffers and workspace fit
  // recorded iterations size their launches for the capacity bucket of
  // their atom and request counts: the workspace is reserved for the buckets
  const bool graphs = o->use_graphs != 0;
  auto ws_atoms = [&](int64_t n) { return graphs ? launch_bucket(n) : n; };
  const int ws_sys = graphs ? (int)launch_bucket(o->max_active) : o->max_active;
  auto need = [&](int64_t n) {
    return fixed + 28ull * (uint64_t)n + model_workspace_bytes(m, ws_atoms(n), ws_sys, true);
  };
  int64_t hi = o->max_batch_atoms > 0 ? o->max_batch_atoms : o->slots;
  hi = std::min<int64_t>(hi, o->slots);
  int64_t lo = 0;
  if (need(hi) <= budget) {
    lo = hi;
  } else {
    while (lo < hi) {  // largest n in [0, hi] with need(n) <= budget
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (need(mid) <= budget) lo = mid; else hi = mid - 1;
    }
  }
  if (lo < 1) return fail(NNP_ENOMEM, "no batch fits the memory budget of %llu bytes", (unsigned long long)budget);

  std::unique_ptr<nnp_server> s(new nnp_server());
  s->model = m;
  s->device = dev;
  s->slots = o->slots;
  s->max_batch = lo;
  s->max_active = o->max_active;
  s->cap = cap;
  s->skin = o->skin;
  s->granted = need(lo);
  s->t0 = now_s();
  s->sched.reset(new Scheduler(o->slots, lo, o->max_active));
  int rc;
  if ((rc = s->store_x.alloc((size_t)o->slots * 12)) || (rc = s->store_s.alloc((size_t)o->slots * 4)) ||
      (rc = s->bx.alloc((size_t)lo * 12)) || (rc = s->bs.alloc((size_t)lo * 4)) ||
      (rc = s->bf.alloc((size_t)lo * 12)) || (rc = s->be.alloc((size_t)o->max_active * 8)) ||
      (rc = s->bsys.alloc((size_t)o->max_active * sizeof(ServeSys))) ||
      (rc = s->bcnt.alloc((size_t)o->max_active * 4)))
    return rc;
  s->n_species = model_species(m);
  if ((rc = nnp_nlist_create(m, o->slots, cap, o->skin, &s->list))) return rc;
  if ((rc = model_reserve_pooled(m, ws_atoms(lo), ws_sys))) {
    nnp_nlist_destroy(s->list);
    s->list = nullptr;
    return rc;
  }
  s->gr.pre = serve_pre;
  s->gr.post = serve_post;
  s->gr.ctx = s.get();
  s->gr.use_graph = graphs;
  if (graphs) {
    s->gr.cache = graph_cache_create();
    // recording needs a stream other than the null stream (default priority)
    hipError_t e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      s->cap_stream = nullptr;
      nnp_server_destroy(s.release());
      return fail(NNP_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    s->gr.capture_stream = s->cap_stream;
  }
  for (auto &it : s->ring) {
    hipError_t e = hipEventCreateWithFlags(&it.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      nnp_server_destroy(s.release());
      return fail(NNP_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  *out = s.release();
  return NNP_OK;
}

extern "C" void nnp_server_destroy(nnp_server *s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  for (auto &it : s->ring)
    if (it.done) {
      if (it.busy) (void)hipEventSynchronize(it.done);
      (void)hipEventDestroy(it.done);
    }
  if (s->list) nnp_nlist_destroy(s->list);
  graph_cache_destroy(s->gr.cache);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  // flags raised by requests that failed alone are the server's business:
  // leave the model's flags clear for its next user
  (void)hipMemset(const_cast<int *>(model_status_word(s->model)), 0, 2 * sizeof(int));
  delete s;
}

extern "C" double nnp_server_clock(const nnp_server *s) { return s ? server_clock(s) : 0.0; }

extern "C" int nnp_server_submit(nnp_server *s, const nnp_request *r, double t_arrival, int64_t *id) {
  if (!s || !r || !id) return fail(NNP_EINVAL, "null argument");
  if (r->n_atoms < 1 || r->n_steps < 1 || !r->coords || !r->species || !(r->sigma >= 0.f))
    return fail(NNP_EINVAL, "bad request");
  for (int a = 0; a < 3; ++a)
    if (!(r->box[a] >= 0.f)) return fail(NNP_EINVAL, "negative box length");
  for (int a = 0; a < r->n_atoms; ++a)
    if (r->species[a] < 0 || r->species[a] >= s->n_species)
      return fail(NNP_ESPECIES, "atom %d: species %d outside the model's %d", a, (int)r->species[a],
                  s->n_species);
  const int64_t rid = s->next_id;
  const double ta = t_arrival >= 0.0 ? t_arrival : server_clock(s);
  if (!s->sched->submit(rid, r->n_atoms, r->n_steps, ta))
    return fail(NNP_EINVAL, "request of %d atoms can never run (pool %lld slots, batch budget %lld atoms)",
                r->n_atoms, (long long)s->slots, (long long)s->max_batch);
  ++s->next_id;
  Request &q = s->reqs[rid];
  q.n = r->n_atoms;
  q.n_steps = r->n_steps;
  memcpy(q.box, r->box, sizeof q.box);
  q.sigma = r->sigma;
  q.seed = r->seed;
  q.coords.assign(r->coords, r->coords + 3 * (size_t)r->n_atoms);
  q.species.assign(r->species, r->species + r->n_atoms);
  q.energy.assign(r->n_steps, 0.0);
  *id = rid;
  return NNP_OK;
}

extern "C" int nnp_server_step(nnp_server *s, void *stream, int64_t *pending) {
  if (!s) return fail(NNP_EINVAL, "null server");
  if (s->sticky) return fail(s->sticky, "an unexpected device flag was raised");
  HIP_TRY(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  int rc = retire_ready(s);
  if (rc) return rc;
  bool launched = false;
  rc = launch_iteration(s, st, &launched);
  if (rc) return rc;
  while ((int)s->inflight.size() >= kDepth || (!launched && !s->inflight.empty())) {
    if ((rc = retire_one(s, true))) return rc;
    if (!launched) break;
  }
  if ((rc = retire_ready(s))) return rc;
  if (pending) *pending = s->sched->queued() + s->sched->active() + (int64_t)s->inflight.size();
  return s->sticky ? fail(s->sticky, "an unexpected device flag was raised") : NNP_OK;
}

extern "C" int nnp_server_drain(nnp_server *s) {
  if (!s) return fail(NNP_EINVAL, "null server");
  while (!s->inflight.empty()) {
    int rc = retire_one(s, true);
    if (rc) return rc;
  }
  return s->sticky ? fail(s->sticky, "an unexpected device flag was raised") : NNP_OK;
}

extern "C" int nnp_server_poll(nnp_server *s, int64_t *ids, int max, int *n) {
  if (!s || !n || (max > 0 && !ids)) return fail(NNP_EINVAL, "null argument");
  const int k = std::min<int>(max, (int)s->ready.size());
  for (int q = 0; q < k; ++q) ids[q] = s->ready[q];
  s->ready.erase(s->ready.begin(), s->ready.begin() + k);
  *n = k;
  return NNP_OK;
}

extern "C" int nnp_server_result(nnp_server *s, int64_t id, double *energies, float *coords, float *forces,
                                 double *times) {
  if (!s) return fail(NNP_EINVAL, "null server");
  const Job *j = s->sched->job(id);
  auto f = s->reqs.find(id);
  if (!j || f == s->reqs.end() || (j->completed < j->n_steps && !j->failed))
    return fail(NNP_EINVAL, "request %lld is not finished or was already collected", (long long)id);
  const Request &r = f->second;
  if (r.error) {
    if (times) {
      times[0] = j->t_arrival;
      times[1] = j->t_admitted;
      times[2] = j->t_done;
    }
    const int err = r.error, mx = r.max_count, steps = j->completed;
    s->reqs.erase(f);
    s->sched->forget(id);
    s->ready.erase(std::remove(s->ready.begin(), s->ready.end(), id), s->ready.end());
    return fail(err, "request %lld stopped after %d steps: a neighbour list of %d entries overflowed the "
                     "capacity of %d", (long long)id, steps, mx, s->cap);
  }
  if (energies) memcpy(energies, r.energy.data(), 8 * r.energy.size());
  if (coords) memcpy(coords, r.last_coords.data(), 4 * r.last_coords.size());
  if (forces) memcpy(forces, r.last_forces.data(), 4 * r.last_forces.size());
  if (times) {
    times[0] = j->t_arrival;
    times[1] = j->t_admitted;
    times[2] = j->t_done;
  }
  s->reqs.erase(f);
  s->sched->forget(id);
  s->ready.erase(std::remove(s->ready.begin(), s->ready.end(), id), s->ready.end());
  return NNP_OK;
}

extern "C" int nnp_server_stats(nnp_server *s, nnp_server_counters *out) {
  if (!s || !out) return fail(NNP_EINVAL, "null argument");
  out->iterations = s->sched->iterations();
  out->atom_evals = s->sched->atom_evals();
  out->queued = s->sched->queued();
  out->active = s->sched->active();
  out->max_batch_atoms = s->max_batch;
  out->max_batch_seen = s->max_batch_seen;
  out->device_bytes = s->granted;
  out->list_builds = 0;
  out->graph_captures = s->gr.captures;
  out->graph_replays = s->gr.replays;
  out->host_launch_s = s->host_s;
  if (s->list) {
    int rc = nnp_nlist_builds(s->list, nullptr, &out->list_builds);
    if (rc) return rc;
  }
  return NNP_OK;
}

// ------------------------------------------------ host-only scheduler ABI

struct nnp_sched {
  Scheduler s;
  std::vector<LaunchItem> last;
  nnp_sched(int64_t slots, int64_t max_batch, int max_active) : s(slots, max_batch, max_active) {}
};

extern "C" int nnp_sched_create(int64_t slots, int64_t max_batch_atoms, int max_active, nnp_sched **out) {
  if (!out) return fail(NNP_EINVAL, "null argument");
  *out = nullptr;
  if (slots < 1 || max_batch_atoms < 1 || max_active < 1) return fail(NNP_EINVAL, "bad scheduler limits");
  *out = new nnp_sched(slots, max_batch_atoms, max_active);
  return NNP_OK;
}

extern "C" void nnp_sched_destroy(nnp_sched *q) { delete q; }

extern "C" int nnp_sched_submit(nnp_sched *q, int64_t id, int n_atoms, int n_steps, double t_arrival) {
  if (!q) return fail(NNP_EINVAL, "null scheduler");
  if (!q->s.submit(id, n_atoms, n_steps, t_arrival))
    return fail(NNP_EINVAL, "request %lld of %d atoms can never run", (long long)id, n_atoms);
  return NNP_OK;
}

extern "C" int nnp_sched_admit(nnp_sched *q, double now, int64_t *ids, int64_t *slots, int max, int *n) {
  if (!q || !n) return fail(NNP_EINVAL, "null argument");
  if (max < 0) return fail(NNP_EINVAL, "negative max");
  // at most `max`, the caller's buffer; the rest stay queued
  const std::vector<int64_t> got = q->s.admit(now, (size_t)max);
  for (size_t k = 0; k < got.size(); ++k) {
    if (ids) ids[k] = got[k];
    if (slots) slots[k] = q->s.job(got[k])->slot;
  }
  *n = (int)got.size();
  return NNP_OK;
}

extern "C" int nnp_sched_launch(nnp_sched *q, int64_t *ids, int64_t *slots, int32_t *n_atoms, int32_t *steps,
                                int max, int *n) {
  if (!q || !n) return fail(NNP_EINVAL, "null argument");
  if (q->s.active() > max) return fail(NNP_EINVAL, "output buffer too small for %lld requests",
                                       (long long)q->s.active());
  std::vector<LaunchItem> items = q->s.launch();
  for (size_t k = 0; k < items.size(); ++k) {
    if (ids) ids[k] = items[k].id;
    if (slots) slots[k] = items[k].slot;
    if (n_atoms) n_atoms[k] = items[k].n_atoms;
    if (steps) steps[k] = items[k].step;
  }
  *n = (int)items.size();
  return NNP_OK;
}

extern "C" int nnp_sched_complete(nnp_sched *q, int64_t id, double now, int *finished) {
  if (!q) return fail(NNP_EINVAL, "null scheduler");
  const Job *j = q->s.job(id);
  if (!j || j->completed >= j->launched) return fail(NNP_EINVAL, "request %lld has no step in flight", (long long)id);
  const bool fin = q->s.complete(id, now);
  if (finished) *finished = fin ? 1 : 0;
  return NNP_OK;
}

extern "C" int nnp_sched_fail(nnp_sched *q, int64_t id, double now) {
  if (!q) return fail(NNP_EINVAL, "null scheduler");
  if (!q->s.fail(id, now)) return fail(NNP_EINVAL, "request %lld is not admitted and unfinished", (long long)id);
  return NNP_OK;
}

extern "C" int nnp_sched_job(nnp_sched *q, int64_t id, double *times, int64_t *slot, int32_t *steps_done) {
  if (!q) return fail(NNP_EINVAL, "null scheduler");
  const Job *j = q->s.job(id);
  if (!j) return fail(NNP_EINVAL, "unknown request %lld", (long long)id);
  if (times) {
    times[0] = j->t_arrival;
    times[1] = j->t_admitted;
    times[2] = j->t_done;
  }
  if (slot) *slot = j->slot;
  if (steps_done) *steps_done = j->completed;
  return NNP_OK;
}

extern "C" int nnp_sched_info(nnp_sched *q, int64_t *info) {
  if (!q || !info) return fail(NNP_EINVAL, "null argument");
  info[0] = q->s.queued();
  info[1] = q->s.active();
  info[2] = q->s.active_atoms();
  info[3] = q->s.free_slots();
  info[4] = q->s.iterations();
  info[5] = q->s.atom_evals();
  return NNP_OK;
}
