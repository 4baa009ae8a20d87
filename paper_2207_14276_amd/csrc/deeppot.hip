// DeepPot-style local-frame descriptor and its gradient (section "DeePMD
// Models"): the neighbours of a centre inside rc, grouped by species and
// ordered nearest first, at most sel[s] of species s kept; each kept
// neighbour fills four features {1/R, x/R, y/R, z/R}, (x, y, z) being its
// coordinates in the centre's local frame.  The frame: e_x along the nearest
// neighbour a, e_y along the part of the second nearest b orthogonal to e_x,
// e_z = e_x x e_y; with one neighbour, or b collinear with a, e_y = e_z = 0.
//
// The neighbour order (and the cutoff test) is an integer decision taken in
// float64 from the caller's float32 coordinates: d = (c_j - c_i) + m L with
// m the lattice image relative to those coordinates, R^2 = (dx dx + dy dy)
// + dz dz, each operation rounded on its own; exact ties go to the smaller
// neighbour index, then the smaller image (x, y, z).  The features use the
// float32 neighbour vector of the packed atom records, as the AEV kernels do.
//
// Forward, one wavefront per centre:
//   1. lane per list entry: per-species counts of the list by ballot (the
//      buckets' capacities);
//   2. again lane per entry: the float64 R^2 and cutoff test, placement of
//      the entries inside the cutoff into per-species buckets in LDS (key,
//      tie, float32 vector, atom index);
//   3. per species bucket, lane per entry: rank = number of bucket entries
//      ahead of it (O(n_s^2 / 64) per lane, all lanes reading the same LDS
//      word at a time); ranks below sel[s] claim a slot; ranks 0 and 1 are
//      the species' frame candidates;
//   4. the two nearest among the candidates give the frame;
//   5. lane per slot: four features, written as one 16-byte (8-byte in
//      bfloat16) store, empty slots as zeros, and the slot's record
//      {d_x, d_y, d_z, j} for the backward (records 0 and 1: the frame's
//      neighbours a and b), one coalesced 16-byte store per lane.
// Backward, one wavefront per centre: lane per slot, reading the slot's
// record (one coalesced load, no neighbour-list or atom gathers), the
// explicit derivative of the slot's features with respect to its vector and
// the frame sums A_c = sum_j (dE/dc_j) d_j / R_j, reduced over the wave; the
// frame terms then reach the axis neighbours a and b.  Global float atomics
// dominated the time of that per-centre form, so forces are summed in LDS
// first: per system for batches of small non-periodic systems (stored once,
// no atomics), per cell of the cell grid otherwise (one set of atomics per
// distinct atom and cell); the per-centre form with atomics remains for the
// caller's pair lists.
#include "internal.h"
#include "wave.h"

namespace nnp {

namespace {

// Slot record of the backward: the neighbour vector and, in w, the
// neighbour's atom index as int bits (-1: empty slot).
__device__ inline float4 slot_record(const float4 &d, int j) { return make_float4(d.x, d.y, d.z, __int_as_float(j)); }

// Per-wave LDS header.
struct DpHead {
  int cnt[8], off[8];                      // valid entries per species, bucket offsets
  int fa, fb, pad0, pad1;                  // bucket positions of the frame neighbours (-1: none)
  ulonglong2 cand[2 * kMaxSpecies + 2];    // each species' two nearest (key, tie)
  int candv[2 * kMaxSpecies + 2];          // their bucket positions (-1: none)
};

__host__ __device__ inline size_t dp_head_bytes() { return (sizeof(DpHead) + 15) / 16 * 16; }
// header, then per list entry: key/tie 16, vector 16, atom index 4; slot table
__host__ __device__ inline size_t dp_lds_bytes(int cap, int n_slots) {
  return dp_head_bytes() + (size_t)cap * (16 + 16 + 4) + ((size_t)n_slots * 4 + 15) / 16 * 16;
}

// Squared distance of the neighbour order, float64, no fused operations:
// the same value whichever compiler contraction rules apply elsewhere.
__device__ inline double dp_key(const float ci[3], const float *cj, int mx, int my, int mz,
                                const double L[3]) {
#pragma clang fp contract(off)
  const double dx = ((double)cj[0] - (double)ci[0]) + (double)mx * L[0];
  const double dy = ((double)cj[1] - (double)ci[1]) + (double)my * L[1];
  const double dz = ((double)cj[2] - (double)ci[2]) + (double)mz * L[2];
  return (dx * dx + dy * dy) + dz * dz;
}

// (key, tie) lexicographic order; R^2 >= 0, so its bits order like the value
__device__ inline bool before(const ulonglong2 &a, const ulonglong2 &b) {
  return a.x < b.x || (a.x == b.x && a.y < b.y);
}

// One list entry of centre i: validity, species, order key and tie.
struct Entry {
  int2 en;
  bool valid;
  int sj;
  ulonglong2 kt;
};

__device__ inline Entry read_entry(int e, int n, const int2 *__restrict__ row, int j0, int n_sys,
                                   const float4 *__restrict__ pos, const float *__restrict__ coords,
                                   const AtomState *__restrict__ state, long long state_j0,
                                   bool wrapped, const int wi[3], const float ci[3],
                                   const double Ld[3], double rc2) {
  Entry r;
  r.en = make_int2(0, 0);
  r.valid = false;
  r.sj = -1;
  r.kt = make_ulonglong2(~0ull, ~0ull);
  if (e >= n) return r;
  r.en = row[e];
  if ((unsigned)r.en.x >= (unsigned)n_sys) return r;
  const int j = j0 + r.en.x;
  r.sj = __float_as_int(pos[j].w);
  if (r.sj < 0) return r;
  int mx, my, mz;
  unpack_image(r.en.y, mx, my, mz);
  if (wrapped) {
    // images refer to the wrapped records; shift them to the caller's frame
    const float4 wj = state[state_j0 + r.en.x].wrap;
    mx += wi[0] - (int)wj.x;
    my += wi[1] - (int)wj.y;
    mz += wi[2] - (int)wj.z;
  }
  const double key = dp_key(ci, coords + 3 * (size_t)j, mx, my, mz, Ld);
  r.valid = key < rc2;
  const unsigned img = ((unsigned)(mx + 512) & 1023u) << 20 | ((unsigned)(my + 512) & 1023u) << 10 |
                       ((unsigned)(mz + 512) & 1023u);
  r.kt = make_ulonglong2((unsigned long long)__double_as_longlong(key),
                         (unsigned long long)(unsigned)r.en.x << 32 | img);
  return r;
}

// Local axes from the float32 vectors (and lengths) of a and b.
struct Frame {
  float ex[3], ey[3], ez[3];
  float ra, nu;  // |d_a|; |u| (0: e_y, e_z undefined)
};

__device__ inline Frame make_frame(bool has_a, const float4 &da, bool has_b, const float4 &db) {
  Frame f;
  for (int k = 0; k < 3; ++k) f.ex[k] = f.ey[k] = f.ez[k] = 0.f;
  f.ra = 1.f;
  f.nu = 0.f;
  if (!has_a) return f;
  f.ra = da.w;
  const float ia = 1.f / da.w;
  f.ex[0] = da.x * ia; f.ex[1] = da.y * ia; f.ex[2] = da.z * ia;
  if (!has_b) return f;
  const float t = db.x * f.ex[0] + db.y * f.ex[1] + db.z * f.ex[2];
  const float u0 = db.x - t * f.ex[0], u1 = db.y - t * f.ex[1], u2 = db.z - t * f.ex[2];
  const float uu = u0 * u0 + u1 * u1 + u2 * u2;
  if (!(uu > 1e-12f * (db.x * db.x + db.y * db.y + db.z * db.z))) return f;
  f.nu = sqrtf(uu);
  const float iu = 1.f / f.nu;
  f.ey[0] = u0 * iu; f.ey[1] = u1 * iu; f.ey[2] = u2 * iu;
  f.ez[0] = f.ex[1] * f.ey[2] - f.ex[2] * f.ey[1];
  f.ez[1] = f.ex[2] * f.ey[0] - f.ex[0] * f.ey[2];
  f.ez[2] = f.ex[0] * f.ey[1] - f.ex[1] * f.ey[0];
  return f;
}

__device__ inline uint16_t bf16_rne(float v) {
  uint32_t a = __float_as_uint(v);
  a += 0x7fffu + ((a >> 16) & 1u);
  return (uint16_t)(a >> 16);
}

template <bool BF16> __device__ inline void store_slot(void *row, int k, float4 f);
template <> __device__ inline void store_slot<false>(void *row, int k, float4 f) { ((float4 *)row)[k] = f; }
template <> __device__ inline void store_slot<true>(void *row, int k, float4 f) {
  uint2 p;
  p.x = (uint32_t)bf16_rne(f.x) | (uint32_t)bf16_rne(f.y) << 16;
  p.y = (uint32_t)bf16_rne(f.z) | (uint32_t)bf16_rne(f.w) << 16;
  ((uint2 *)row)[k] = p;
}

}  // namespace

template <int WPB, bool BF16>
__global__ void __launch_bounds__(WPB * kWave)
k_dp_fwd(const float4 *__restrict__ pos, const float *__restrict__ coords,
         const AtomState *__restrict__ state, const int *__restrict__ sys_of,
         const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
         const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
         void *__restrict__ G, int ldg, int N, DpConst c, float4 *__restrict__ rec) {
  extern __shared__ float4 lds4[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int i = blockIdx.x * WPB + wave;
  if (i >= N) return;
  const int r = row_of_atom[i];
  if (r < 0) return;  // outside a caller's mask: no network row
  char *base = (char *)lds4 + (size_t)wave * dp_lds_bytes(cap, c.n_slots);
  DpHead *h = (DpHead *)base;
  ulonglong2 *bkt = (ulonglong2 *)(base + dp_head_bytes());
  float4 *bd = (float4 *)(bkt + cap);
  int *bj = (int *)(bd + cap);
  int *smap = bj + cap;

  const SysDesc &d = sys[sys_of[i]];
  const int n = min(nbr_cnt[d.state_off + (i - d.atom_off)], cap);
  const float4 pi = pos[i];
  const float L[3] = {d.L[0], d.L[1], d.L[2]};
  const double Ld[3] = {(double)d.L[0], (double)d.L[1], (double)d.L[2]};
  const int j0 = d.atom_off, n_sys = d.n;
  const int2 *row = nbr + nbr_row(d, i, cap);
  const float ci[3] = {coords[3 * (size_t)i], coords[3 * (size_t)i + 1], coords[3 * (size_t)i + 2]};
  const bool wrapped = d.periodic != 0;
  int wi[3] = {0, 0, 0};
  if (wrapped) {
    const float4 w = state[d.state_off + (i - d.atom_off)].wrap;
    wi[0] = (int)w.x; wi[1] = (int)w.y; wi[2] = (int)w.z;
  }

  // 1. list entries per species: bucket capacities (the cutoff test in step 2
  //    may drop some; buckets then keep unused space at their ends)
  int cnt[kMaxSpecies];
#pragma unroll
  for (int s = 0; s < kMaxSpecies; ++s) cnt[s] = 0;
  for (int b = 0; b < n; b += kWave) {
    const int e = b + lane;
    int sj = -1;
    if (e < n) {
      const int2 en = row[e];
      if ((unsigned)en.x < (unsigned)n_sys) sj = __float_as_int(pos[j0 + en.x].w);
    }
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) cnt[s] += __popcll(__ballot(sj == s));
  }
  int off[kMaxSpecies];
  {
    int o = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) { off[s] = o; o += cnt[s]; }
  }
  if (lane == 0) {
    h->fa = -1;
    h->fb = -1;
  }
  if (lane < 2 * kMaxSpecies + 2) {
    h->cand[lane] = make_ulonglong2(~0ull, ~0ull);
    h->candv[lane] = -1;
  }
  for (int k = lane; k < c.n_slots; k += kWave) smap[k] = -1;

  // 2. species buckets
  {
    int run[kMaxSpecies];
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) run[s] = 0;
    for (int b = 0; b < n; b += kWave) {
      const int e = b + lane;
      const Entry x = read_entry(e, n, row, j0, n_sys, pos, coords, state, d.state_off, wrapped, wi, ci,
                                 Ld, c.rc2);
      int at = 0;
#pragma unroll
      for (int s = 0; s < kMaxSpecies; ++s) {
        const unsigned long long m = __ballot(x.valid && x.sj == s);
        if (x.valid && x.sj == s) at = off[s] + run[s] + (int)lanes_below(m);
        run[s] += __popcll(m);
      }
      if (x.valid) {
        bkt[at] = x.kt;
        bd[at] = entry_vec(pi, pos[j0 + x.en.x], x.en.y, L);
        bj[at] = j0 + x.en.x;
      }
    }
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) cnt[s] = run[s];   // the entries inside the cutoff
  }
  wave_lds_sync();

  // 3. rank inside each species bucket
  for (int s = 0; s < c.S; ++s) {
    const int cs = cnt[s], os = off[s], sel = c.sel[s], so = c.soff[s];
    for (int vb = 0; vb < cs; vb += kWave) {
      const int q = vb + lane;
      const bool act = q < cs;
      const ulonglong2 me = act ? bkt[os + q] : make_ulonglong2(~0ull, ~0ull);
      int rank = 0;
      for (int t = 0; t < cs; ++t) rank += before(bkt[os + t], me) ? 1 : 0;
      if (act && rank < sel) smap[so + rank] = os + q;
      if (act && rank < 2) {
        h->cand[2 * s + rank] = me;
        h->candv[2 * s + rank] = os + q;
      }
    }
  }
  wave_lds_sync();

  // 4. the frame: the two nearest among the species' two nearest
  if (lane < 2 * c.S) {
    const ulonglong2 me = h->cand[lane];
    const int v = h->candv[lane];
    int g = 0;
    for (int t = 0; t < 2 * c.S; ++t) g += before(h->cand[t], me) ? 1 : 0;
    if (v >= 0 && g == 0) h->fa = v;
    if (v >= 0 && g == 1) h->fb = v;
  }
  wave_lds_sync();
  const int fa = h->fa, fb = h->fb;
  const Frame f = make_frame(fa >= 0, fa >= 0 ? bd[fa] : make_float4(0.f, 0.f, 0.f, 1.f), fb >= 0,
                             fb >= 0 ? bd[fb] : make_float4(0.f, 0.f, 0.f, 1.f));

  // 5. features and the slot records
  void *Grow = (char *)G + (size_t)r * ldg * (BF16 ? 2 : 4);
  float4 *rrow = rec ? rec + (size_t)i * c.ldm : nullptr;
  if (rrow && lane < 2) {
    const int v = lane == 0 ? fa : fb;
    rrow[lane] = v >= 0 ? slot_record(bd[v], bj[v]) : slot_record(make_float4(0.f, 0.f, 0.f, 0.f), -1);
  }
  for (int k = lane; k < c.n_slots; k += kWave) {
    const int v = smap[k];
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (v >= 0) {
      const float4 dv = bd[v];
      const float ir = 1.f / dv.w;
      out.x = ir;
      out.y = (dv.x * f.ex[0] + dv.y * f.ex[1] + dv.z * f.ex[2]) * ir;
      out.z = (dv.x * f.ey[0] + dv.y * f.ey[1] + dv.z * f.ey[2]) * ir;
      out.w = (dv.x * f.ez[0] + dv.y * f.ez[1] + dv.z * f.ez[2]) * ir;
    }
    store_slot<BF16>(Grow, k, out);
    if (rrow)
      rrow[2 + k] = v >= 0 ? slot_record(bd[v], bj[v]) : slot_record(make_float4(0.f, 0.f, 0.f, 0.f), -1);
  }
}

// Backward of centre i (one wavefront, row r of dE/dG): the explicit terms
// of its slots, the frame terms, and its virial share.  add(j, x, y, z) takes
// a contribution to the force on atom j; every lane may call it.
template <class Add>
__device__ inline void dp_centre_bwd(int i, int lane, int r, const float *__restrict__ dG, int ldg,
                                     const DpConst &c, const float4 *__restrict__ rec,
                                     float *__restrict__ W_atom, Add &&add) {
  const float4 *rrow = rec + (size_t)i * c.ldm;
  const float4 ra = rrow[0], rb = rrow[1];
  const int ja = __float_as_int(ra.w), jb = __float_as_int(rb.w);
  float4 da = make_float4(ra.x, ra.y, ra.z, 1.f), db = make_float4(rb.x, rb.y, rb.z, 1.f);
  if (ja >= 0) da.w = fast_sqrt(da.x * da.x + da.y * da.y + da.z * da.z);
  if (jb >= 0) db.w = fast_sqrt(db.x * db.x + db.y * db.y + db.z * db.z);
  const Frame f = make_frame(ja >= 0, da, jb >= 0, db);
  const float4 *g4 = (const float4 *)(dG + (size_t)r * ldg);

  // explicit terms, lane per slot; A[3c + k] = sum_j (dE/dG_{j,1+c}) d_j[k] / R_j
  float A[9], fi[3], vir[9];
  for (int q = 0; q < 9; ++q) A[q] = vir[q] = 0.f;
  fi[0] = fi[1] = fi[2] = 0.f;
  for (int k = lane; k < c.n_slots; k += kWave) {
    const float4 rk = rrow[2 + k];
    const int j = __float_as_int(rk.w);
    if (j < 0) continue;
    const float4 gs = g4[k];
    const float dvv[3] = {rk.x, rk.y, rk.z};
    const float ir = 1.f / fast_sqrt(rk.x * rk.x + rk.y * rk.y + rk.z * rk.z);
    const float cx = rk.x * f.ex[0] + rk.y * f.ex[1] + rk.z * f.ex[2];
    const float cy = rk.x * f.ey[0] + rk.y * f.ey[1] + rk.z * f.ey[2];
    const float cz = rk.x * f.ez[0] + rk.y * f.ez[1] + rk.z * f.ez[2];
    // d(1/R)/dd = -d/R^3, d(c/R)/dd = e_c/R - c d/R^3 (axes held fixed)
    const float s = (gs.x + gs.y * cx + gs.z * cy + gs.w * cz) * ir * ir * ir;
    float gd[3];
    for (int a = 0; a < 3; ++a) {
      gd[a] = -s * dvv[a] + (gs.y * f.ex[a] + gs.z * f.ey[a] + gs.w * f.ez[a]) * ir;
      A[a] += gs.y * ir * dvv[a];
      A[3 + a] += gs.z * ir * dvv[a];
      A[6 + a] += gs.w * ir * dvv[a];
      fi[a] += gd[a];
    }
    add(j, -gd[0], -gd[1], -gd[2]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) vir[3 * a + b] -= dvv[a] * gd[b];
  }
  for (int q = 0; q < 9; ++q) A[q] = wave_sum(A[q]);
  for (int q = 0; q < 9; ++q) vir[q] = wave_sum(vir[q]);
  for (int a = 0; a < 3; ++a) fi[a] = wave_sum(fi[a]);

  // frame terms: e_x = d_a/|d_a|, e_y = u/|u| with u = (I - e_x e_x^T) d_b,
  // e_z = e_x x e_y; every lane holds the reduced sums
  if (ja >= 0) {
    float Bx[3] = {A[0], A[1], A[2]};
    float gb[3] = {0.f, 0.f, 0.f};
    const float dbv[3] = {db.x, db.y, db.z}, dav[3] = {da.x, da.y, da.z};
    if (f.nu > 0.f) {
      const float *Az = A + 6;
      float By[3] = {A[3], A[4], A[5]};
      // through e_z: dE/de_x += e_y x A_z, dE/de_y += A_z x e_x
      Bx[0] += f.ey[1] * Az[2] - f.ey[2] * Az[1];
      Bx[1] += f.ey[2] * Az[0] - f.ey[0] * Az[2];
      Bx[2] += f.ey[0] * Az[1] - f.ey[1] * Az[0];
      By[0] += Az[1] * f.ex[2] - Az[2] * f.ex[1];
      By[1] += Az[2] * f.ex[0] - Az[0] * f.ex[2];
      By[2] += Az[0] * f.ex[1] - Az[1] * f.ex[0];
      const float byy = By[0] * f.ey[0] + By[1] * f.ey[1] + By[2] * f.ey[2];
      const float iu = 1.f / f.nu;
      float C[3];
      for (int a = 0; a < 3; ++a) C[a] = (By[a] - byy * f.ey[a]) * iu;
      const float cx = C[0] * f.ex[0] + C[1] * f.ex[1] + C[2] * f.ex[2];
      const float bx = dbv[0] * f.ex[0] + dbv[1] * f.ex[1] + dbv[2] * f.ex[2];
      for (int a = 0; a < 3; ++a) {
        gb[a] = C[a] - cx * f.ex[a];
        Bx[a] += -cx * dbv[a] - bx * C[a];
      }
    }
    const float bxx = Bx[0] * f.ex[0] + Bx[1] * f.ex[1] + Bx[2] * f.ex[2];
    const float ia = 1.f / f.ra;
    float ga[3];
    for (int a = 0; a < 3; ++a) ga[a] = (Bx[a] - bxx * f.ex[a]) * ia;
    for (int a = 0; a < 3; ++a) {
      fi[a] += ga[a] + gb[a];
      for (int b = 0; b < 3; ++b) vir[3 * a + b] -= dav[a] * ga[b] + dbv[a] * gb[b];
    }
    if (lane == 0) add(ja, -ga[0], -ga[1], -ga[2]);
    if (lane == 1 && f.nu > 0.f) add(jb, -gb[0], -gb[1], -gb[2]);
  }
  if (lane == 2) add(i, fi[0], fi[1], fi[2]);
  if (lane < 9) {
    float v = vir[0];
    for (int q = 1; q < 9; ++q) v = lane == q ? vir[q] : v;
    W_atom[(size_t)9 * i + lane] = v;
  }
}

// Any batch: one wavefront per centre, forces by float atomics.
template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_dp_bwd(const int *__restrict__ row_of_atom, const float *__restrict__ dG, int ldg, int N, DpConst c,
         const float4 *__restrict__ rec, float *__restrict__ F, float *__restrict__ W_atom) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int i = blockIdx.x * WPB + wave;
  if (i >= N) return;
  const int r = row_of_atom[i];
  if (r < 0) {  // outside a caller's mask: no energy, no virial share
    if (lane < 9) W_atom[(size_t)9 * i + lane] = 0.f;
    return;
  }
  dp_centre_bwd(i, lane, r, dG, ldg, c, rec, W_atom, [&](int j, float x, float y, float z) {
    atomicAdd(&F[3 * (size_t)j], x);
    atomicAdd(&F[3 * (size_t)j + 1], y);
    atomicAdd(&F[3 * (size_t)j + 2], z);
  });
}

// Batches of small non-periodic systems (every neighbour inside the centre's
// own system): one workgroup per system, its waves taking the system's
// centres in turn; the system's forces are summed in LDS (64-bit fixed
// point, integer atomics) and stored once, with no global atomics.
template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_dp_bwd_sys(const SysDesc *__restrict__ sys, const int *__restrict__ row_of_atom,
             const float *__restrict__ dG, int ldg, DpConst c, const float4 *__restrict__ rec,
             float *__restrict__ F, float *__restrict__ W_atom) {
  __shared__ unsigned long long facc[3 * kSmallSystem];
  const SysDesc &d = sys[blockIdx.x];
  const int n = d.n, a0 = d.atom_off;
  for (int t = threadIdx.x; t < 3 * n; t += WPB * kWave) facc[t] = 0ull;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  for (int il = wave; il < n; il += WPB) {
    const int i = a0 + il;
    const int r = row_of_atom[i];
    if (r < 0) {
      if (lane < 9) W_atom[(size_t)9 * i + lane] = 0.f;
      continue;
    }
    dp_centre_bwd(i, lane, r, dG, ldg, c, rec, W_atom, [&](int j, float x, float y, float z) {
      unsigned long long *p = facc + 3 * (j - a0);
      atomicAdd(p, (unsigned long long)to_fix(x));
      atomicAdd(p + 1, (unsigned long long)to_fix(y));
      atomicAdd(p + 2, (unsigned long long)to_fix(z));
    });
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 3 * n; t += WPB * kWave) F[3 * (size_t)a0 + t] = from_fix((long long)facc[t]);
}

template <bool BF16>
static void dp_fwd_t(const float4 *pos, const float *coords, const AtomState *state, const int *sys_of,
                     const SysDesc *sys, const int2 *nbr, const int *nbr_cnt, int cap,
                     const int *row_of_atom, void *G, int ldg, int N, const DpConst &c, float4 *rec,
                     int wpb, hipStream_t st) {
  const size_t lds = dp_lds_bytes(cap, c.n_slots) * wpb;
  const unsigned grid = (unsigned)((N + wpb - 1) / wpb);
  if (wpb == 4)
    k_dp_fwd<4, BF16><<<grid, 4 * kWave, lds, st>>>(pos, coords, state, sys_of, sys, nbr, nbr_cnt, cap,
                                                    row_of_atom, G, ldg, N, c, rec);
  else if (wpb == 2)
    k_dp_fwd<2, BF16><<<grid, 2 * kWave, lds, st>>>(pos, coords, state, sys_of, sys, nbr, nbr_cnt, cap,
                                                    row_of_atom, G, ldg, N, c, rec);
  else
    k_dp_fwd<1, BF16><<<grid, kWave, lds, st>>>(pos, coords, state, sys_of, sys, nbr, nbr_cnt, cap,
                                                row_of_atom, G, ldg, N, c, rec);
}

// Waves per workgroup: the preference (1, 2 or 4) when its LDS fits in
// 64 KB, else one.
void launch_dp_fwd(const float4 *pos, const float *coords, const AtomState *state, const int *sys_of,
                   const SysDesc *sys, const int2 *nbr, const int *nbr_cnt, int cap,
                   const int *row_of_atom, void *G, bool g_bf16, int ldg, int N, const DpConst &c,
                   float4 *rec, int wpb_pref, hipStream_t st) {
  if (N <= 0) return;
  int wpb = 1;
  if ((wpb_pref == 2 || wpb_pref == 4) && dp_lds_bytes(cap, c.n_slots) * wpb_pref <= 64 * 1024) wpb = wpb_pref;
  if (g_bf16) dp_fwd_t<true>(pos, coords, state, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, N, c, rec, wpb, st);
  else dp_fwd_t<false>(pos, coords, state, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, N, c, rec, wpb, st);
}

// Systems on a cell grid: one workgroup per cell, its waves taking the cell's
// centres in turn.  The centres of one cell share most of their neighbours,
// so their force contributions are first summed in an LDS hash table keyed
// by atom index (open addressing, 64-bit fixed-point sums) and each distinct
// atom receives one set of float atomics per cell instead of one per
// contribution.  A contribution that finds the table full goes straight to
// global memory.
constexpr int kMinCellGroups = 256;
constexpr int kHashBits = 11;
constexpr int kHashSlots = 1 << kHashBits;   // 2048 atoms; a cell's neighbourhood holds ~700

template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_dp_bwd_cells(const int *__restrict__ cell_start, const int *__restrict__ cell_atoms,
               const int *__restrict__ row_of_atom, const float *__restrict__ dG, int ldg, DpConst c,
               const float4 *__restrict__ rec, float *__restrict__ F, float *__restrict__ W_atom) {
  __shared__ int hkey[kHashSlots];
  __shared__ unsigned long long hval[3 * kHashSlots];
  const int b = cell_start[blockIdx.x], e = cell_start[blockIdx.x + 1];
  if (b == e) return;  // the whole workgroup leaves together
  for (int t = threadIdx.x; t < kHashSlots; t += WPB * kWave) {
    hkey[t] = -1;
    hval[3 * t] = hval[3 * t + 1] = hval[3 * t + 2] = 0ull;
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  for (int p = b + wave; p < e; p += WPB) {
    const int i = cell_atoms[p];
    const int r = row_of_atom[i];
    if (r < 0) {
      if (lane < 9) W_atom[(size_t)9 * i + lane] = 0.f;
      continue;
    }
    dp_centre_bwd(i, lane, r, dG, ldg, c, rec, W_atom, [&](int j, float x, float y, float z) {
      unsigned h = ((unsigned)j * 2654435761u) >> (32 - kHashBits);
      for (int probe = 0; probe < kHashSlots; ++probe) {
        int k = hkey[h];
        if (k == -1) k = atomicCAS(&hkey[h], -1, j);  // -1: this lane claimed the slot
        if (k == -1 || k == j) {
          atomicAdd(&hval[3 * h], (unsigned long long)to_fix(x));
          atomicAdd(&hval[3 * h + 1], (unsigned long long)to_fix(y));
          atomicAdd(&hval[3 * h + 2], (unsigned long long)to_fix(z));
          return;
        }
        h = (h + 1) & (kHashSlots - 1);
      }
      atomicAdd(&F[3 * (size_t)j], x);
      atomicAdd(&F[3 * (size_t)j + 1], y);
      atomicAdd(&F[3 * (size_t)j + 2], z);
    });
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHashSlots; t += WPB * kWave) {
    const int j = hkey[t];
    if (j < 0) continue;
    atomicAdd(&F[3 * (size_t)j], from_fix((long long)hval[3 * t]));
    atomicAdd(&F[3 * (size_t)j + 1], from_fix((long long)hval[3 * t + 1]));
    atomicAdd(&F[3 * (size_t)j + 2], from_fix((long long)hval[3 * t + 2]));
  }
}

// The per-centre backward uses no LDS: four waves per workgroup unless asked
// otherwise.  With small_systems (every system non-periodic with at most
// kSmallSystem atoms) the per-system form runs instead, eight waves per
// system; with a cell grid (cell_start non-null) of at least one cell per
// compute unit the per-cell form, eight waves per cell (fewer cells leave
// most of the chip idle: the 2,001-atom water box has 64).
void launch_dp_bwd(const SysDesc *sys, int n_sys, bool small_systems, const int *cell_start,
                   const int *cell_atoms, int n_cells, const int *row_of_atom, const float *dG, int ldg, int N,
                   const DpConst &c, const float4 *rec, float *F, float *W_atom, int wpb_pref, hipStream_t st) {
  if (N <= 0) return;
  if (small_systems) {
    k_dp_bwd_sys<8><<<n_sys, 8 * kWave, 0, st>>>(sys, row_of_atom, dG, ldg, c, rec, F, W_atom);
    return;
  }
  if (cell_start && n_cells >= kMinCellGroups) {
    k_dp_bwd_cells<8><<<n_cells, 8 * kWave, 0, st>>>(cell_start, cell_atoms, row_of_atom, dG, ldg, c, rec, F,
                                                     W_atom);
    return;
  }
  const int wpb = (wpb_pref == 1 || wpb_pref == 2) ? wpb_pref : 4;
  const unsigned grid = (unsigned)((N + wpb - 1) / wpb);
  if (wpb == 4)
    k_dp_bwd<4><<<grid, 4 * kWave, 0, st>>>(row_of_atom, dG, ldg, N, c, rec, F, W_atom);
  else if (wpb == 2)
    k_dp_bwd<2><<<grid, 2 * kWave, 0, st>>>(row_of_atom, dG, ldg, N, c, rec, F, W_atom);
  else
    k_dp_bwd<1><<<grid, kWave, 0, st>>>(row_of_atom, dG, ldg, N, c, rec, F, W_atom);
}

}  // namespace nnp
