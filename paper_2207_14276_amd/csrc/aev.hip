// Atomic environment vectors and their gradient (section "ANI models":
// cosine cutoff, radial and angular symmetry functions).
//
// One wavefront per centre atom; for calls of several systems the waves take
// the centres of the largest systems first (wave_atom), so that no costly
// centre starts last.  The centre's neighbour entries (its list row, or for
// small systems without a list the atoms of its system) are re-derived from
// the packed atom records and sorted by neighbour species into LDS with wave
// ballots.  Then
//   radial:  lanes = 16 radial shifts x 4 neighbour slots, one species block
//            at a time, reduced across the 4 slots with lane shuffles;
//   angular (forward): the species-pair blocks in passes of 64 pair slots;
//            a pass holds a 64-pair piece of a large block, or the rest of
//            one block followed by whole smaller blocks, each padded to a
//            multiple of 8 slots:
//            (A) lane per slot: the pair geometry (cos and sin of the angle,
//                the 4 radial Gaussians of the mean distance times the
//                cutoff product) is computed once and staged in a per-wave
//                LDS scratch;
//            (B) lanes = 8 angle shifts x 8 slots, block by block: each lane
//                evaluates the cosine power of its angle shift for a pair
//                and accumulates the 4 radial-shift products; accumulators
//                are reduced across the 8 slots once a block's last pair is
//                done.
//            Blocks without a pair are written as zeros directly.
//   angular (backward): the pairs of all species-pair blocks form one
//            stream, one pair per lane; a lane evaluates all 8 angle shifts
//            of its pair against the block's dE/dG values (read from the
//            centre's row, which stays in the L1/L2 caches), recomputes the
//            angular cutoff of both legs, differentiates through cos, sin,
//            R_j and R_k, and accumulates dE/dd_j and dE/dd_k per neighbour
//            entry in the wave's LDS (float64 atomics, in a fixed order).
//            Forces then go to the accumulators in 64-bit fixed point.
// The backward keeps its LDS per wave near 7 KB (5 waves per SIMD at a
// neighbour capacity of 128) by recomputing the angular cutoffs and reading
// dE/dG from cache; its VALU issue, not memory, sets its time, so every
// instruction saved in the per-pair loop counts.
#include "internal.h"
#include "wave.h"

namespace nnp {

constexpr float kPi = 3.14159265358979323846f;

__device__ inline float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float fast_log2(float x) { return __builtin_amdgcn_logf(x); }


// q = u / n and r = u mod n for 0 <= u < 2^23 through a float reciprocal
// (rn within an ulp of 1/n): the estimate is off by at most one, corrected
// by selects.
__device__ inline int fdivmod(int u, int n, float rn, int &r) {
  int q = (int)((float)u * rn);
  int m = u - q * n;
  const bool hi = m >= n, lo = m < 0;
  q = hi ? q + 1 : (lo ? q - 1 : q);
  r = hi ? m - n : (lo ? m + n : m);
  return q;
}

// Wave-uniform per-species counts and offsets of the sorted lists.
struct Lists {
  int cR[8], oR[8];
  int cA[8], oA[8];
};

// LDS layout of one wave's lists (cap entries each), pair-block table and
// pair scratch.
constexpr int kPairPass = kWave;  // neighbour pairs staged per pass
constexpr int kMaxBlocks = kMaxSpecies * (kMaxSpecies + 1) / 2;
constexpr int kMaxAng = kMaxBlocks * kAngBlock;  // 896 angular features

struct WaveLds {
  Lists *ls;       // per-species counts and offsets (wave-uniform)
  float2 *tGeo;    // pair scratch: cos, sin                      (forward)
  float4 *tF2;     // pair scratch: radial Gaussians of Rbar times
                   // fc_j fc_k                                     (forward)
  float4 *rD;      // radial: unit vector d / R and R
  float *rFc;      // radial: fc_rad(R)          (forward)
  float2 *rF2;     // fc(R) and fc'(R): radial cutoff, then (angular entries)
                   // the angular cutoff once the radial stage is done (backward)
  int *rJ;         // radial: neighbour index     (backward)
  double *rG;      // radial: dE/dd accumulators, float64 (backward, 3 per entry)
  int *aIdx;       // angular: position in the radial arrays  (backward)
  unsigned short *aIdx16;  // the same, 16-bit       (forward)
  float *aFc;      // angular: fc_ang(R)          (forward)
};

// Per-wave LDS bytes (a multiple of 16).  Forward entry: rD 16, rFc 4,
// aIdx16 2 (the array padded to 16 bytes), aFc 4: 4,992 bytes per wave at a
// capacity of 128, so that 8 waves per SIMD fit.  Backward entry: rD 16,
// rG 24, rF2 8, rJ 4, aIdx 4; the backward reads the centre's dE/dG row from
// global memory (it stays in the L1/L2 caches) and keeps the angular cutoff
// in the radial cutoff's slots: 7,296 bytes per wave at a capacity of 128
// (5 waves per SIMD).
__host__ __device__ inline size_t aidx16_bytes(int cap) { return ((size_t)cap * 2 + 15) / 16 * 16; }

template <bool BWD>
__host__ __device__ inline size_t wave_lds_bytes(int cap) {
  return sizeof(Lists) + (BWD ? (size_t)cap * (16 + 24 + 4 + 4 + 4 + 4)
                              : (size_t)kPairPass * (8 + 16) +
                                    (size_t)cap * (16 + 4 + 4) + aidx16_bytes(cap));
}

template <bool BWD>
__device__ inline WaveLds carve(char *base, int cap) {
  WaveLds w{};
  char *p = base;
  w.ls = (Lists *)p; p += sizeof(Lists);
  if (BWD) {
    w.rD = (float4 *)p; p += (size_t)cap * 16;
    w.rG = (double *)p; p += (size_t)cap * 24;
    w.rF2 = (float2 *)p; p += (size_t)cap * 8;
    w.rJ = (int *)p; p += (size_t)cap * 4;
    w.aIdx = (int *)p; p += (size_t)cap * 4;
  } else {
    w.tGeo = (float2 *)p; p += (size_t)kPairPass * 8;
    w.tF2 = (float4 *)p; p += (size_t)kPairPass * 16;
    w.rD = (float4 *)p; p += (size_t)cap * 16;
    w.rFc = (float *)p; p += (size_t)cap * 4;
    w.aIdx16 = (unsigned short *)p; p += aidx16_bytes(cap);
    w.aFc = (float *)p; p += (size_t)cap * 4;
  }
  return w;
}

// Lane b (< S (S + 1) / 2) describes species-pair block b of the centre's
// angular pairs, in the upper-triangle order of (sa, sb) that is also the
// feature order: its pair count T and the unrank fields of its two lists
// (a pair is addressed as (x, y), x in the longer species list of length n1,
// y in the shorter of length n2; a same-species block uses the one list for
// both; the angular term is symmetric in its two neighbours): oxy = offsets
// of the x and y lists (16 bits each), ns = n1 | n2 << 16 | same << 31,
// r2 = 1 / n2 (a hardware reciprocal: fdivmod corrects the quotient).
// Other lanes get T = 0.
__device__ inline void block_words(int lane, const Lists &ls, int S, int &bT, int &bOxy, int &bNs, float &bR2) {
  bT = 0;
  bOxy = 0;
  bNs = 0;
  bR2 = 1.f;
  if (lane < S * (S + 1) / 2) {
    int sa = 0, rem = lane;
#pragma unroll
    for (int s = 0; s < kMaxSpecies - 1; ++s)
      if (sa == s && rem >= S - s) { rem -= S - s; sa = s + 1; }
    const int sb = sa + rem;
    const int na = ls.cA[sa], nb = ls.cA[sb], oa = ls.oA[sa], ob = ls.oA[sb];
    const bool same = sa == sb;
    bT = same ? na * (na - 1) / 2 : na * nb;
    const bool a_long = na >= nb;
    const int n1 = max(na, nb), n2 = min(na, nb);
    bOxy = (a_long ? oa : ob) | ((a_long ? ob : oa) << 16);
    bNs = n1 | (n2 << 16) | (same ? (int)0x80000000u : 0);
    bR2 = fast_rcp((float)max(n2, 1));
  }
}

// List positions (ax, ay) of pair u of a block (ns and r2 as in
// block_words), with u = q n2 + y.  Two species: x = (y + q) mod n1, q < n1.
// One species of n entries (n1 = n2 = n): q < n / 2 and the pair is
// {y, (y + q + 1) mod n}, q + 1 being its distance around the list, so that
// every unordered pair comes once (for even n the last row q = n / 2 - 1
// holds only y < n / 2).  Either way y + q (+ 1) < 2 n1, and neighbouring
// lanes take different entries of both lists (their LDS adds to an entry's
// accumulators do not pile up on one address).
__device__ inline void unrank(int u, int ns, float r2, int oxy, int &ax, int &ay) {
  const int n1 = ns & 0xffff, n2 = (ns >> 16) & 0x7fff;
  int y;
  const int q = fdivmod(u, n2, r2, y);
  int x = y + q + (ns < 0 ? 1 : 0);
  x = x >= n1 ? x - n1 : x;
  ax = (oxy & 0xffff) + x;
  ay = ((oxy >> 16) & 0xffff) + y;
}

// One neighbour entry of a centre: the atom (index within the system's
// records at j0), its species and the vector d (R in w); false for an entry
// past the row or whose stored atom index is not below n_sys (a reused list
// applied to a different system), which is never dereferenced.  self >= 0:
// no list; entry e is the system's atom e (n = n_sys), the centre (local
// index self) excluded.
__device__ __attribute__((always_inline)) inline bool load_entry(int e, int n, const int2 *__restrict__ ent,
                                                                 int self, int j0, int n_sys,
                                                                 const float4 *__restrict__ pos,
                                                                 const float4 &pi, const float L[3], int &sj, int &j,
                                                                 float4 &d) {
  int2 en = make_int2(0, 0);
  if (self >= 0) en = make_int2(e, pack_image(0, 0, 0));
  else if (e < n) en = ent[e];
  const bool v = e < n && (unsigned)en.x < (unsigned)n_sys && en.x != self;
  sj = -1;
  j = 0;
  d = make_float4(0.f, 0.f, 0.f, 1e30f);
  if (v) {
    j = j0 + en.x;
    const float4 pj = pos[j];
    d = entry_vec(pi, pj, en.y, L);
    sj = __float_as_int(pj.w);
  }
  return v;
}

// Builds the species-sorted radial list (R < rc_r) and angular list
// (R < rc_a, a subset) of centre i in LDS from its neighbour row, or (self
// >= 0) from all atoms of its system, keeping those a list would hold (R^2
// below rc_r^2 as the list build tests it).  Two passes over the entries:
// per-species counts by ballot, then placement.  Rows of up to 128 entries
// (the common case) are loaded once and kept in registers for both passes;
// longer rows are loaded again.  Per-species tallies live in registers
// (loops over the species slots are fully unrolled; species without an
// entry in a chunk are skipped) and the wave-uniform result is published
// in LDS.
template <bool BWD>
__device__ inline void fill_lists(int lane, int n, const int2 *__restrict__ ent, int self, int j0, int n_sys,
                                  const float4 *__restrict__ pos, const float4 &pi,
                                  const float L[3], const AevConst &c, WaveLds &w) {
  const int S = c.S;
  const bool cached = n <= 2 * kWave;  // wave-uniform
  const float rc2 = c.rc_r * c.rc_r;
  int sj0 = -1, sj1 = -1, jj0 = 0, jj1 = 0;
  float4 d0 = make_float4(0.f, 0.f, 0.f, 1e30f), d1 = d0;
  if (cached) {
    load_entry(lane, n, ent, self, j0, n_sys, pos, pi, L, sj0, jj0, d0);
    if (n > kWave) load_entry(kWave + lane, n, ent, self, j0, n_sys, pos, pi, L, sj1, jj1, d1);
  }
  int cR[kMaxSpecies], cA[kMaxSpecies];
#pragma unroll
  for (int s = 0; s < kMaxSpecies; ++s) { cR[s] = 0; cA[s] = 0; }
  for (int b = 0; b < n; b += kWave) {
    int sj, j;
    float4 d;
    if (cached) {  // the entry of this lane in the chunk starting at b
      const bool first = b == 0;
      sj = first ? sj0 : sj1;
      j = first ? jj0 : jj1;
      d = first ? d0 : d1;
    } else {
      load_entry(b + lane, n, ent, self, j0, n_sys, pos, pi, L, sj, j, d);
    }
    const bool inR = sj >= 0 && d.w < c.rc_r && (self < 0 || d.x * d.x + d.y * d.y + d.z * d.z < rc2),
               inA = inR && d.w < c.rc_a;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      cR[s] += __popcll(__ballot(inR && sj == s));
      cA[s] += __popcll(__ballot(inA && sj == s));
    }
  }
  int pR[kMaxSpecies], pA[kMaxSpecies];
  {
    int oR = 0, oA = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      pR[s] = oR; oR += cR[s];
      pA[s] = oA; oA += cA[s];
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      w.ls->cR[s] = s < S ? cR[s] : 0; w.ls->oR[s] = pR[s];
      w.ls->cA[s] = s < S ? cA[s] : 0; w.ls->oA[s] = pA[s];
    }
  }
  const float kr = kPi / c.rc_r, ka = kPi / c.rc_a;
  (void)ka;
  for (int b = 0; b < n; b += kWave) {
    int sj, j;
    float4 d;
    if (cached) {  // the entry of this lane in the chunk starting at b
      const bool first = b == 0;
      sj = first ? sj0 : sj1;
      j = first ? jj0 : jj1;
      d = first ? d0 : d1;
    } else {
      load_entry(b + lane, n, ent, self, j0, n_sys, pos, pi, L, sj, j, d);
    }
    const bool inR = sj >= 0 && d.w < c.rc_r && (self < 0 || d.x * d.x + d.y * d.y + d.z * d.z < rc2),
               inA = inR && d.w < c.rc_a;
    // slots of this lane's entry in the two lists (selects per species;
    // the stores below are then issued once, not once per species)
    int q = 0, qa = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      const unsigned long long mR = __ballot(inR && sj == s);
      if (!mR) continue;  // (the angular list is a subset of the radial one)
      const unsigned long long mA = __ballot(inA && sj == s);
      if (sj == s) {
        q = pR[s] + (int)lanes_below(mR);
        qa = pA[s] + (int)lanes_below(mA);
      }
      pR[s] += __popcll(mR);
      pA[s] += __popcll(mA);
    }
    if (inR) {
      float sn, cs;
      __sincosf(kr * d.w, &sn, &cs);
      // the pair geometry and the gradients need only the direction and R
      const float ir = fast_rcp(d.w);
      w.rD[q] = make_float4(d.x * ir, d.y * ir, d.z * ir, d.w);
      if (BWD) {
        w.rF2[q] = make_float2(0.5f * cs + 0.5f, -0.5f * kr * sn);
        w.rJ[q] = j;
      } else {
        w.rFc[q] = 0.5f * cs + 0.5f;
      }
    }
    if (inA) {
      if (BWD) w.aIdx[qa] = q;
      else w.aIdx16[qa] = (unsigned short)q;
      if (!BWD) w.aFc[qa] = 0.5f * __cosf(ka * d.w) + 0.5f;
    }
  }
}

// Element k of a small constant table for a lane-dependent k, by selects
// (a dynamically indexed kernel argument would go through scratch memory).
template <int N> __device__ inline float pick(const float (&t)[N], int k) {
  float v = t[0];
#pragma unroll
  for (int q = 1; q < N; ++q) v = k == q ? t[q] : v;
  return v;
}

__device__ inline uint32_t bf16_pair(float lo, float hi) {
  uint32_t a = __float_as_uint(lo), b = __float_as_uint(hi);
  a += 0x7fffu + ((a >> 16) & 1u);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (a >> 16) | (b & 0xffff0000u);
}

// Eight consecutive features (row offset k, a multiple of 8) from LDS to the
// feature row in one 16-byte (bfloat16) or two 16-byte (float32) stores.
template <bool BF16> __device__ inline void store8(void *row, int k, const float *v);
template <> __device__ inline void store8<true>(void *row, int k, const float *v) {
  uint4 o;
  o.x = bf16_pair(v[0], v[1]); o.y = bf16_pair(v[2], v[3]);
  o.z = bf16_pair(v[4], v[5]); o.w = bf16_pair(v[6], v[7]);
  *(uint4 *)((uint16_t *)row + k) = o;
}
template <> __device__ inline void store8<false>(void *row, int k, const float *v) {
  float4 *d = (float4 *)((float *)row + k);
  d[0] = make_float4(v[0], v[1], v[2], v[3]);
  d[1] = make_float4(v[4], v[5], v[6], v[7]);
}

// One feature (row offset k) to the feature row, rounded to bfloat16 the
// same way as bf16_pair.  The lanes of a wave that store together cover
// contiguous features, so the stores combine into full segments.
template <bool BF16> __device__ inline void store1(void *row, int k, float v);
template <> __device__ inline void store1<true>(void *row, int k, float v) {
  uint32_t a = __float_as_uint(v);
  a += 0x7fffu + ((a >> 16) & 1u);
  ((uint16_t *)row)[k] = (uint16_t)(a >> 16);
}
template <> __device__ inline void store1<false>(void *row, int k, float v) { ((float *)row)[k] = v; }

// Bit p of x (p < 32) to bits 2 p and 2 p + 1.
__device__ inline unsigned long long spread_pairs(unsigned long long x) {
  x &= 0xffffffffull;
  x = (x | (x << 16)) & 0x0000ffff0000ffffull;
  x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
  x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x | (x << 1);
}
// The row mask's halves: a radial block is one 16-column half, an angular
// block two, and all of them fit in 64 bits.
static_assert(kNShfRad == 16 && kAngBlock == 32, "row mask halves");
static_assert(kMaxSpecies + kMaxSpecies * (kMaxSpecies + 1) <= 64, "row mask width");

template <int WPB, bool BF16>
__global__ void __launch_bounds__(WPB * kWave)
k_aev_fwd(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
          const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
          const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
          void *__restrict__ G, int ldg, unsigned long long *__restrict__ row_mask,
          const int *__restrict__ wave_atom, int *__restrict__ status, Live N_, AevConst c) {
  extern __shared__ float4 lds4[];
  const int N = N_.get();
  // the wave index is uniform across the wave: keep it (and the centre's
  // index, descriptors and row pointers) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int wv = blockIdx.x * WPB + wave;
  const int i = wave_atom && wv < N ? __builtin_amdgcn_readfirstlane(wave_atom[wv]) : wv;
  // an atom without a network row (outside a caller's mask) is skipped
  const bool live = i < N && row_of_atom[i] >= 0;
  WaveLds w = carve<false>((char *)lds4 + wave * wave_lds_bytes<false>(cap), cap);
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  float L[3] = {0.f, 0.f, 0.f};
  int n = 0, j0 = 0, n_sys = 0, self = -1;
  const int2 *row = nbr;
  if (live) {
    const SysDesc &d = sys[sys_of[i]];
    n_sys = d.n;
    pi = pos[i];
    L[0] = d.L[0]; L[1] = d.L[1]; L[2] = d.L[2];
    j0 = d.atom_off;
    if (nbr) {
      n = min(nbr_cnt[d.state_off + (i - d.atom_off)], cap);
      row = nbr + nbr_row(d, i, cap);
    } else {
      n = n_sys;  // no list: the system's atoms
      self = i - d.atom_off;
    }
  }
  fill_lists<false>(lane, n, row, self, j0, n_sys, pos, pi, L, c, w);
  __syncthreads();
  if (!live) return;
  const Lists &ls = *w.ls;
  // without a list, the largest neighbour count (what the list build
  // records) goes to status[1]: the current value is read here and compared
  // at the end, so that the wave does not wait for it
  int nb_cnt = 0, nb_max = 0;
  if (status) {
    for (int s = 0; s < c.S; ++s) nb_cnt += ls.cR[s];
    nb_max = __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const int r_i = row_of_atom[i];
  void *Grow = (char *)G + (size_t)r_i * ldg * (BF16 ? 2 : 4);

  // radial: G[16 s + m] = scale * sum_j exp(-eta (R - Rs_m)^2) fc(R)
  // lanes = 16 shifts x 4 neighbour slots (slot fastest)
  {
    const int m = lane >> 2, slot = lane & 3;
    const float shf = pick(c.shf_r, m);
    const float keta = -c.eta_r * 1.4426950408889634f;
    for (int s = 0; s < c.S; ++s) {
      float acc = 0.f;
      const int o = ls.oR[s];
      const int cnt = ls.cR[s];
      // no branch per entry: slots past the end re-read the last entry
      // and add it with a zero weight
      for (int e0 = 0; e0 < cnt; e0 += 4) {
        const int e = e0 + slot;
        const int q = o + min(e, cnt - 1);
        const float t = w.rD[q].w - shf;
        acc += fast_exp2(keta * t * t) * (e < cnt ? w.rFc[q] : 0.f);
      }
      acc = sum4(acc);
      if (slot == 0) store1<BF16>(Grow, s * kNShfRad + m, acc * c.scale);
    }
  }

  // angular: G[rad_len + 32 p + 8 r + a] = sum over pairs {j, k} of
  //   2^(1-zeta) (1 + cos(theta - theta_a))^zeta exp(-eta (Rbar - Rs_r)^2) fc_j fc_k
  {
    const int a = lane >> 3, t0 = lane & 7;  // phase B: 8 angle shifts x 8 pairs (pair fastest)
    // y = (1 + cos(theta - theta_a)) / 2 in [0, 1] (clamped by its own FMA),
    // so that 2^(1-zeta) (1 + cos)^zeta = 2 y^zeta = 2^(zeta log2 y + 1)
    const float hcz = pick(c.hcz, a), hsz = pick(c.hsz, a);
    const float keta = -c.eta_a * 1.4426950408889634f;
    // lane b: species-pair block b (block_words)
    const int n_blk = c.S * (c.S + 1) / 2;
    int bT, bOxy, bNs;
    float bR2;
    block_words(lane, ls, c.S, bT, bOxy, bNs, bR2);
    const unsigned long long nonempty = __ballot(bT > 0);
    // the row's record of its possibly non-zero halves: radial species with
    // an entry, species pairs with a pair
    if (row_mask) {
      const unsigned long long radial = __ballot(lane < c.S && ls.cR[min(lane, kMaxSpecies - 1)] > 0);
      if (lane == 0) row_mask[r_i] = radial | spread_pairs(nonempty) << c.S;
    }
    // blocks without a pair of their two species are zero: written in one
    // pass of 16-byte stores over the angular part of the row
    {
      constexpr int kChunksPerBlock = kAngBlock * (BF16 ? 2 : 4) / 16;
      uint4 *ang = (uint4 *)((char *)Grow + (size_t)c.rad_len * (BF16 ? 2 : 4));
      for (int k = lane; k < n_blk * kChunksPerBlock; k += kWave)
        if (!((nonempty >> (k / kChunksPerBlock)) & 1ull)) ang[k] = make_uint4(0u, 0u, 0u, 0u);
    }
    // Passes of 64 pair slots.  A block with more than 64 pairs left fills
    // a pass on its own; otherwise the pass takes the rest of the block and
    // then whole following blocks while they fit, each padded to a multiple
    // of 8 slots, so that every group of 8 slots belongs to one block.
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
    unsigned long long pending = nonempty;
    int u = 0;  // pairs of the first pending block done by earlier passes
    while (pending) {
      const int q = __builtin_ctzll(pending);
      const int Tq = __builtin_amdgcn_readlane(bT, q);
      // this lane's slot: block fields, pair index within the block, count
      int l_oxy = __builtin_amdgcn_readlane(bOxy, q);
      int l_ns = __builtin_amdgcn_readlane(bNs, q);
      float l_r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bR2), q));
      int l_u = u + lane, l_T = Tq;
      unsigned long long in_pass = 1ull << q;
      const bool finish = Tq - u <= kPairPass;
      int used = kPairPass;  // slots taken by the pass's blocks
      if (finish) {
        used = (Tq - u + 7) & ~7;
        unsigned long long rest = pending & (pending - 1);
        while (rest) {
          const int q2 = __builtin_ctzll(rest);
          const int T2 = __builtin_amdgcn_readlane(bT, q2);
          const int g2 = (T2 + 7) & ~7;
          if (used + g2 > kPairPass) break;
          if (lane >= used) {
            l_oxy = __builtin_amdgcn_readlane(bOxy, q2);
            l_ns = __builtin_amdgcn_readlane(bNs, q2);
            l_r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bR2), q2));
            l_u = lane - used;
            l_T = T2;
          }
          used += g2;
          in_pass |= 1ull << q2;
          rest &= rest - 1;
        }
      }
      // (A) lane per pair slot; padding slots (and slots past the pass's
      // blocks) repeat a valid pair with a zero cutoff product
      {
        const bool valid = lane < used && l_u < l_T;
        const int tt = min(l_u, l_T - 1);
        int qj, qk;
        unrank(tt, l_ns, l_r2, l_oxy, qj, qk);
        const float4 dj = w.rD[w.aIdx16[qj]], dk = w.rD[w.aIdx16[qk]];  // unit vectors, R
        const float cosv = dj.x * dk.x + dj.y * dk.y + dj.z * dk.z;
        const float cx = dj.y * dk.z - dj.z * dk.y;
        const float cy = dj.z * dk.x - dj.x * dk.z;
        const float cz = dj.x * dk.y - dj.y * dk.x;
        const float sinv = fast_sqrt(cx * cx + cy * cy + cz * cz);
        const float fcc = valid ? w.aFc[qj] * w.aFc[qk] : 0.f;
        const float Rbar = 0.5f * (dj.w + dk.w);
        const float u0 = Rbar - c.shf_a[0], u1 = Rbar - c.shf_a[1];
        const float u2 = Rbar - c.shf_a[2], u3 = Rbar - c.shf_a[3];
        w.tGeo[lane] = make_float2(cosv, sinv);
        w.tF2[lane] = make_float4(fcc * fast_exp2(keta * u0 * u0), fcc * fast_exp2(keta * u1 * u1),
                                  fcc * fast_exp2(keta * u2 * u2), fcc * fast_exp2(keta * u3 * u3));
      }
      wave_lds_sync();
      // (B) per block of the pass, its groups of 8 slots two at a time; a
      // block's accumulators are reduced across the 8 pairs and stored once
      // its last pair is done
      {
        int g = 0;  // first group of the block in the pass
        unsigned long long blocks = in_pass;
        while (blocks) {
          const int k = __builtin_ctzll(blocks);
          blocks &= blocks - 1;
          const int Tk = __builtin_amdgcn_readlane(bT, k);
          const int ng = k == q ? (finish ? (Tq - u + 7) >> 3 : kPairPass / 8) : (Tk + 7) >> 3;
          const int gend = g + ng;
          for (; g + 2 <= gend; g += 2) {
            const int q0 = 8 * g + t0, q1 = q0 + 8;
            const float2 geo0 = w.tGeo[q0], geo1 = w.tGeo[q1];
            const float4 f20 = w.tF2[q0], f21 = w.tF2[q1];
            const float y0 = __builtin_amdgcn_fmed3f(fmaf(geo0.x, hcz, fmaf(geo0.y, hsz, 0.5f)), 0.f, 1.f);
            const float y1 = __builtin_amdgcn_fmed3f(fmaf(geo1.x, hcz, fmaf(geo1.y, hsz, 0.5f)), 0.f, 1.f);
            const float v0 = fast_exp2(c.zeta * fast_log2(y0) + 1.0f);
            const float v1 = fast_exp2(c.zeta * fast_log2(y1) + 1.0f);
            acc0 += v0 * f20.x; acc0 += v1 * f21.x;
            acc1 += v0 * f20.y; acc1 += v1 * f21.y;
            acc2 += v0 * f20.z; acc2 += v1 * f21.z;
            acc3 += v0 * f20.w; acc3 += v1 * f21.w;
          }
          if (g < gend) {
            const int q0 = 8 * g + t0;
            const float2 geo = w.tGeo[q0];
            const float4 f2 = w.tF2[q0];
            const float y = __builtin_amdgcn_fmed3f(fmaf(geo.x, hcz, fmaf(geo.y, hsz, 0.5f)), 0.f, 1.f);
            const float v = fast_exp2(c.zeta * fast_log2(y) + 1.0f);
            acc0 += v * f2.x; acc1 += v * f2.y; acc2 += v * f2.z; acc3 += v * f2.w;
            ++g;
          }
          if (k != q || finish) {
            // sums over the 8 slot lanes of each angle shift, halving the
            // values in flight at each step: the two quads of the 8 lanes
            // swap halves (r 0, 1 stay low, r 2, 3 high), then the lane
            // pairs of a quad, then neighbours add; lane t0 ends with
            // r = 2 (t0 >> 2) + ((t0 >> 1) & 1)
            const bool hi = t0 >= 4, b1 = (t0 >> 1) & 1;
            const float A = (hi ? acc2 : acc0) + dpp<0x141>(hi ? acc0 : acc2);  // row_half_mirror
            const float B = (hi ? acc3 : acc1) + dpp<0x141>(hi ? acc1 : acc3);
            float C = (b1 ? B : A) + dpp<0x4E>(b1 ? A : B);                      // quad_perm [2,3,0,1]
            C += dpp<0xB1>(C);                                                   // quad_perm [1,0,3,2]
            if (!(t0 & 1)) {
              const int r = 2 * (t0 >> 2) + ((t0 >> 1) & 1);
              store1<BF16>(Grow, c.rad_len + k * kAngBlock + kNShfZ * r + a, C);
            }
            acc0 = acc1 = acc2 = acc3 = 0.f;
          }
        }
      }
      wave_lds_sync();
      if (finish) {
        pending &= ~in_pass;
        u = 0;
      } else {
        u += kPairPass;
      }
    }
  }
  if (status && lane == 0 && nb_cnt > nb_max) atomicMax(status + 1, nb_cnt);
}

// Where the force contributions of a centre go.  Forces accumulate in 64-bit
// fixed point (fixed.h) in the buffer Ffix[N][3], which the caller clears
// first and converts to float32 afterwards: integer sums do not depend on the
// order in which waves add into them, so forces come out the same bit for
// bit whatever else the batch holds.  Atom j of system d accumulates in slot
// j + fix_shift(d) = d.order_off + (j - d.atom_off): the systems in the
// order their centres are launched, so that the waves running together add
// into neighbouring slots (scattered slots made these device atomics
// several times slower).
//   SinkGlobal: device-scope integer atomics straight into Ffix;
//   SinkSys:    an LDS table of one system's atoms (index j - atom_off),
//               added into Ffix once per workgroup;
//   SinkHash:   an LDS hash table keyed by atom index (open addressing,
//               linear probing), added into Ffix once per workgroup; an atom
//               that finds no free slot within kBwdProbe probes goes
//               straight to Ffix.
struct SinkGlobal {
  unsigned long long *F;
  int shift;  // fix_shift of the system
  __device__ inline void add(int j, long long x, long long y, long long z) const {
    unsigned long long *p = F + 3 * (size_t)(j + shift);
    atomicAdd(p, (unsigned long long)x);
    atomicAdd(p + 1, (unsigned long long)y);
    atomicAdd(p + 2, (unsigned long long)z);
  }
};
struct SinkSys {
  unsigned long long *tab;
  int off;
  __device__ inline void add(int j, long long x, long long y, long long z) const {
    unsigned long long *p = tab + 3 * (j - off);
    atomicAdd(p, (unsigned long long)x);
    atomicAdd(p + 1, (unsigned long long)y);
    atomicAdd(p + 2, (unsigned long long)z);
  }
};
constexpr int kBwdHashBits = 9;
constexpr int kBwdHash = 1 << kBwdHashBits;  // slots: a cell's neighbourhood holds ~300-450 atoms
constexpr int kBwdProbe = 32;
constexpr int kBwdMinCells = 512;  // cells of a grid for the per-cell form
constexpr size_t kBwdStaticLds = 64;  // bytes kept for static LDS of the grouped forms
struct SinkHash {
  int *key;
  unsigned long long *val;
  unsigned long long *F;
  int shift;  // fix_shift of the system
  __device__ inline void add(int j, long long x, long long y, long long z) const {
    unsigned h = ((unsigned)j * 2654435761u) >> (32 - kBwdHashBits);
    for (int probe = 0; probe < kBwdProbe; ++probe) {
      int k = key[h];
      if (k == -1) k = atomicCAS(&key[h], -1, j);  // -1: this lane claimed the slot
      if (k == -1 || k == j) {
        unsigned long long *p = val + 3 * h;
        atomicAdd(p, (unsigned long long)x);
        atomicAdd(p + 1, (unsigned long long)y);
        atomicAdd(p + 2, (unsigned long long)z);
        return;
      }
      h = (h + 1) & (kBwdHash - 1);
    }
    SinkGlobal{F, shift}.add(j, x, y, z);
  }
};

// Backward of centre i by one wave (wave-uniform i; no workgroup barrier, so
// waves of one workgroup may work on different centres): dE/dd of every
// radial entry from the radial and angular terms, the centre's virial row
// W_atom[i] = -sum d (x) dE/dd, and its force contributions through sink:
// -dE/dd onto each neighbour, the sum of dE/dd onto the centre.
template <class Sink>
__device__ inline void bwd_centre(int i, int lane, const float4 *__restrict__ pos, const int *__restrict__ sys_of,
                                  const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
                                  const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
                                  const float *__restrict__ dG, int ldg, const AevConst &c,
                                  float *__restrict__ W_atom, WaveLds &w, const Sink &sink) {
  // an atom without a network row (outside a caller's mask) is skipped; its
  // virial share is zero
  const int r_i = row_of_atom[i];
  if (r_i < 0) {
    if (lane < 9) W_atom[(size_t)9 * i + lane] = 0.f;
    return;
  }
  const SysDesc &d = sys[sys_of[i]];
  const int n_sys = d.n;
  // no list (nbr null): the system's atoms
  const int n = nbr ? min(nbr_cnt[d.state_off + (i - d.atom_off)], cap) : n_sys;
  const int self = nbr ? -1 : i - d.atom_off;
  const float4 pi = pos[i];
  const float L[3] = {d.L[0], d.L[1], d.L[2]};
  const int j0 = d.atom_off;
  const int2 *row = nbr ? nbr + nbr_row(d, i, cap) : nbr;
  fill_lists<true>(lane, n, row, self, j0, n_sys, pos, pi, L, c, w);
  wave_lds_sync();
  const Lists &ls = *w.ls;
  const float *g = dG + (size_t)r_i * ldg;
  int nR = 0;
  for (int s = 0; s < c.S; ++s) nR += ls.cR[s];
  // radial, lane per neighbour entry: with t_m = R - Rs_m and
  // e_m = exp(-eta t_m^2), dE/dR = scale (fc' sum_m g_m e_m - 2 eta fc
  // sum_m g_m e_m t_m), g being the dE/dG values of the entry's species;
  // dE/dd = dE/dR d / R.  This stage is the first writer of the dE/dd
  // accumulators.
  {
    const float keta = -c.eta_r * 1.4426950408889634f;
    for (int e = lane; e < nR; e += kWave) {
      int sp = 0;
#pragma unroll
      for (int s = 1; s < kMaxSpecies; ++s) sp += e >= ls.oR[s] ? 1 : 0;
      const float4 d = w.rD[e];
      const float2 fc = w.rF2[e];
      const float4 *gs = (const float4 *)(g + sp * kNShfRad);
      float A = 0.f, B = 0.f;
#pragma unroll
      for (int h = 0; h < kNShfRad / 4; ++h) {
        const float4 gv = gs[h];
        const float gm[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float t = d.w - c.shf_r[4 * h + k];
          const float ge = gm[k] * fast_exp2(keta * t * t);
          A += ge;
          B += ge * t;
        }
      }
      const float dEdR = c.scale * (fc.y * A - 2.0f * c.eta_r * fc.x * B);
      double *gg = w.rG + 3 * e;
      gg[0] = (double)(dEdR * d.x); gg[1] = (double)(dEdR * d.y); gg[2] = (double)(dEdR * d.z);
    }
  }
  wave_lds_sync();

  // angular cutoff of every angular entry, into its radial cutoff slot (the
  // radial stage above was the last reader of those)
  {
    const float ka = kPi / c.rc_a;
    int nA = 0;
    for (int s = 0; s < c.S; ++s) nA += ls.cA[s];
    for (int e = lane; e < nA; e += kWave) {
      const int q = w.aIdx[e];
      float sn, cs;
      __sincosf(ka * w.rD[q].w, &sn, &cs);
      w.rF2[q] = make_float2(0.5f * cs + 0.5f, -0.5f * ka * sn);
    }
  }
  wave_lds_sync();

  // angular: lane per neighbour pair over the pair stream of all blocks
  // (the blocks' pairs one after another, in feature order)
  {
    const float *gA = g + c.rad_len;
    // lane b: species-pair block b, with the first pair of the block in the
    // stream (an exclusive prefix sum of the counts over the lanes)
    const int n_blk = c.S * (c.S + 1) / 2;
    int bT, bOxy, bNs;
    float bR2;
    block_words(lane, ls, c.S, bT, bOxy, bNs, bR2);
    int bStart = bT;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {  // n_blk <= 28: the first 32 lanes hold every block
      const int y = __shfl_up(bStart, d, 32);
      if ((lane & 31) >= d) bStart += y;
    }
    const int P = __builtin_amdgcn_readlane(bStart, n_blk - 1);
    bStart -= bT;
    const float zm1 = c.zeta - 1.0f;
    const float keta = -c.eta_a * 1.4426950408889634f;
    const float m2eta = -2.0f * c.eta_a;
    // the non-empty block holding the pass's first pair (wave-uniform);
    // the block searches visit non-empty blocks only
    const unsigned long long nonempty = __ballot(bT > 0);
    int qb = nonempty ? __builtin_ctzll(nonempty) : 0;
    for (int base = 0; base < P; base += kPairPass) {
      for (unsigned long long m = nonempty & (~0ull << (qb + 1)); m; m &= m - 1) {
        const int r = __builtin_ctzll(m);
        if (__builtin_amdgcn_readlane(bStart, r) > base) break;
        qb = r;
      }
      const bool valid = base + lane < P;
      const int t = min(base + lane, P - 1);
      // this lane's block: the last non-empty one starting at or before its
      // pair; the pass's blocks are few, their starts wave-uniform
      int p = qb;
      for (unsigned long long m = nonempty & (~0ull << (qb + 1)); m; m &= m - 1) {
        const int r = __builtin_ctzll(m);
        const int sr = __builtin_amdgcn_readlane(bStart, r);
        if (sr >= base + kPairPass) break;
        p = t >= sr ? r : p;
      }
      const int pa = p << 2;
      const int l_oxy = __builtin_amdgcn_ds_bpermute(pa, bOxy);
      const int l_ns = __builtin_amdgcn_ds_bpermute(pa, bNs);
      const float l_r2 = __int_as_float(__builtin_amdgcn_ds_bpermute(pa, __float_as_int(bR2)));
      const int l_start = __builtin_amdgcn_ds_bpermute(pa, bStart);
      int aj, ak;
      unrank(t - l_start, l_ns, l_r2, l_oxy, aj, ak);
      const int qj = w.aIdx[aj], qk = w.aIdx[ak];
      const float4 dj = w.rD[qj], dk = w.rD[qk];      // unit vectors u, v and R
      const float2 cj2 = w.rF2[qj], ck2 = w.rF2[qk];  // angular fc and fc'
      const float cosv = dj.x * dk.x + dj.y * dk.y + dj.z * dk.z;
      const float cx = dj.y * dk.z - dj.z * dk.y;
      const float cy = dj.z * dk.x - dj.x * dk.z;
      const float cz = dj.x * dk.y - dj.y * dk.x;
      const float sinv = fast_sqrt(cx * cx + cy * cy + cz * cz);
      const float Rbar = 0.5f * (dj.w + dk.w);
      float f2[kNShfAng], ur[kNShfAng];
#pragma unroll
      for (int r = 0; r < kNShfAng; ++r) {
        ur[r] = Rbar - c.shf_a[r];
        f2[r] = fast_exp2(keta * ur[r] * ur[r]);
      }
      // dE/dG of this block: gv[r][a] at gA[32 p + 8 r + a] (global, cached).
      // With p1 = 2^(1-zeta) x^(zeta-1) and f1 = p1 x (x = 1 + cos(theta -
      // theta_a)), the pair's terms are f1 f2[r] fc_j fc_k, so
      //   dE/dx_a   = zeta p1 A_a fc_j fc_k,  A_a = sum_r gv[r][a] f2[r]
      //   dE/dRbar  = sum_r f2'[r] H_r fc_j fc_k,  dE/d(fc_j fc_k) = sum_r f2[r] H_r,
      //   H_r = sum_a gv[r][a] f1_a.
      const float4 *gv = (const float4 *)(gA + p * kAngBlock);
      float dcos = 0.f, dsin = 0.f, H[kNShfAng] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float gq[kNShfAng][4];
#pragma unroll
        for (int r = 0; r < kNShfAng; ++r) {
          const float4 v = gv[2 * r + h];
          gq[r][0] = v.x; gq[r][1] = v.y; gq[r][2] = v.z; gq[r][3] = v.w;
        }
#pragma unroll
        for (int aa = 0; aa < 4; ++aa) {
          const int a = 4 * h + aa;
          // y = x / 2 in [0, 1] (clamped by its own FMA); p1 = y^(zeta-1)
          const float y = __builtin_amdgcn_fmed3f(fmaf(cosv, c.hcz[a], fmaf(sinv, c.hsz[a], 0.5f)), 0.f, 1.f);
          const float p1 = fast_exp2(zm1 * fast_log2(y));
          float A = gq[0][aa] * f2[0];
#pragma unroll
          for (int r = 1; r < kNShfAng; ++r) A += gq[r][aa] * f2[r];
          const float s1 = p1 * A;
          dcos += s1 * c.hcz[a];  // half of dE/dcos: doubled below
          dsin += s1 * c.hsz[a];
          const float f1h = p1 * y;  // f1 / 2: H holds half its value
#pragma unroll
          for (int r = 0; r < kNShfAng; ++r) H[r] += gq[r][aa] * f1h;
        }
      }
      if (valid) {
        float dfc = 0.f, dbar = 0.f;
#pragma unroll
        for (int r = 0; r < kNShfAng; ++r) {
          const float t = f2[r] * H[r];
          dfc += t;
          dbar += ur[r] * t;
        }
        const float fj = cj2.x, fk = ck2.x;
        const float fcc = fj * fk;
        const float zf = 2.0f * c.zeta * fcc;  // the halved cos / sin constants
        dcos *= zf;
        dsin *= zf;
        dbar *= m2eta * fcc;  // via Rbar (dRbar/dR = 1/2, H halved), for each of R_j and R_k
        dfc += dfc;           // H halved
        const float dRj = dbar + dfc * cj2.y * fk;
        const float dRk = dbar + dfc * fj * ck2.y;
        // with c = cos, s = sin of the angle and u, v the unit vectors of
        // the legs j, k: d c / d dj = (v - c u) / Rj and d s / d dj =
        // -(c / s) (v - c u) / Rj (likewise for dk with u and v swapped),
        // so dE/d dj = bj v + (dE/dRj - bj c) u with bj = (dE/dc -
        // dE/ds c / s) / Rj.  Where s vanishes (collinear legs) the sine's
        // term is dropped.
        const float beta = dcos - (sinv > 1e-12f ? dsin * cosv * fast_rcp(sinv) : 0.f);
        const float bj = beta * fast_rcp(dj.w), bk = beta * fast_rcp(dk.w);
        const float uj = dRj - bj * cosv, uk = dRk - bk * cosv;
        // float64 LDS atomics: the wave's own region, so the adds to an
        // entry happen in one fixed order (program order, then lane order
        // within an instruction) and the sums are the same on every call
        double *gj = w.rG + 3 * qj;
        double *gk = w.rG + 3 * qk;
        atomicAdd(gj + 0, (double)(bj * dk.x + uj * dj.x));
        atomicAdd(gj + 1, (double)(bj * dk.y + uj * dj.y));
        atomicAdd(gj + 2, (double)(bj * dk.z + uj * dj.z));
        atomicAdd(gk + 0, (double)(bk * dj.x + uk * dk.x));
        atomicAdd(gk + 1, (double)(bk * dj.y + uk * dk.y));
        atomicAdd(gk + 2, (double)(bk * dj.z + uk * dk.z));
      }
    }
    wave_lds_sync();
  }

  // scatter: -dE/dd onto each neighbour, the sum onto the centre (fixed
  // point), per-centre virial -sum d (x) dE/dd
  {
    float fi0 = 0.f, fi1 = 0.f, fi2 = 0.f;
    float vir[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) vir[q] = 0.f;
    for (int e = lane; e < nR; e += kWave) {
      const float4 ur = w.rD[e];  // unit vector and R
      const float4 dv = make_float4(ur.x * ur.w, ur.y * ur.w, ur.z * ur.w, ur.w);
      const float gx = (float)w.rG[3 * e], gy = (float)w.rG[3 * e + 1], gz = (float)w.rG[3 * e + 2];
      sink.add(w.rJ[e], -to_fix(gx), -to_fix(gy), -to_fix(gz));
      fi0 += gx; fi1 += gy; fi2 += gz;
      vir[0] -= dv.x * gx; vir[1] -= dv.x * gy; vir[2] -= dv.x * gz;
      vir[3] -= dv.y * gx; vir[4] -= dv.y * gy; vir[5] -= dv.y * gz;
      vir[6] -= dv.z * gx; vir[7] -= dv.z * gy; vir[8] -= dv.z * gz;
    }
    fi0 = wave_sum(fi0);
    fi1 = wave_sum(fi1);
    fi2 = wave_sum(fi2);
#pragma unroll
    for (int q = 0; q < 9; ++q) vir[q] = wave_sum(vir[q]);
    if (lane == 0) sink.add(i, to_fix(fi0), to_fix(fi1), to_fix(fi2));
    if (lane < 9) {
      float v = vir[0];
#pragma unroll
      for (int q = 1; q < 9; ++q) v = lane == q ? vir[q] : v;
      W_atom[(size_t)9 * i + lane] = v;
    }
  }
  // the next centre of this wave rewrites the lists
  wave_lds_sync();
}

// Per-centre form (caller pair lists, small cell grids): one wave per centre,
// forces by device atomics.
template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_aev_bwd(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
          const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
          const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
          const float *__restrict__ dG, int ldg, Live N, AevConst c, unsigned long long *__restrict__ Ffix,
          float *__restrict__ W_atom, const int *__restrict__ wave_atom) {
  extern __shared__ float4 lds4[];
  // the wave index is uniform across the wave: keep it (and the centre's
  // index, descriptors and row pointers) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int wv = blockIdx.x * WPB + wave;
  if (wv >= N.get()) return;
  // the centre of this wave (the costliest systems' centres first)
  const int i = wave_atom ? __builtin_amdgcn_readfirstlane(wave_atom[wv]) : wv;
  WaveLds w = carve<true>((char *)lds4 + wave * wave_lds_bytes<true>(cap), cap);
  const SysDesc &d = sys[sys_of[i]];
  bwd_centre(i, lane, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, c, W_atom, w,
             SinkGlobal{Ffix, fix_shift(d)});
}

// Next centre of a workgroup's group for the calling wave (an LDS counter:
// waves that finish early take more centres).
__device__ inline int next_centre(int *counter, int lane) {
  int p = 0;
  if (lane == 0) p = atomicAdd(counter, 1);
  return __builtin_amdgcn_readfirstlane(p);
}

// Per-system form (batches of small non-periodic systems): a workgroup takes
// a group of consecutive centres of one system (groups[b] = {first centre,
// count}); the system's forces are summed in an LDS table and added into
// Ffix once.
template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_aev_bwd_sys(const int2 *__restrict__ groups, const float4 *__restrict__ pos, const int *__restrict__ sys_of,
              const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
              const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
              const float *__restrict__ dG, int ldg, AevConst c, unsigned long long *__restrict__ Ffix,
              float *__restrict__ W_atom, Live n_groups) {
  extern __shared__ float4 lds4[];
  __shared__ int counter;
  if ((int)blockIdx.x >= n_groups.get()) return;  // the whole workgroup leaves together
  const int2 gr = groups[blockIdx.x];
  const SysDesc &d = sys[sys_of[gr.x]];
  const int off = d.atom_off, n3 = 3 * d.n;
  unsigned long long *tab = (unsigned long long *)((char *)lds4 + WPB * wave_lds_bytes<true>(cap));
  for (int t = threadIdx.x; t < n3; t += WPB * kWave) tab[t] = 0ull;
  if (threadIdx.x == 0) counter = 0;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  WaveLds w = carve<true>((char *)lds4 + wave * wave_lds_bytes<true>(cap), cap);
  const SinkSys sink{tab, off};
  for (int p = next_centre(&counter, lane); p < gr.y; p = next_centre(&counter, lane))
    bwd_centre(gr.x + p, lane, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, c, W_atom, w, sink);
  __syncthreads();
  for (int t = threadIdx.x; t < n3; t += WPB * kWave) {
    const unsigned long long v = tab[t];
    if (v) atomicAdd(Ffix + 3 * (size_t)d.order_off + t, v);
  }
}

// Per-cell form (cell grids): a workgroup takes the centres of one cell;
// they share most of their neighbours, whose forces are summed in an LDS hash
// table and added into Ffix once per cell.
template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_aev_bwd_cells(const int *__restrict__ cell_start, const int *__restrict__ cell_atoms,
                const float4 *__restrict__ pos, const int *__restrict__ sys_of,
                const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
                const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
                const float *__restrict__ dG, int ldg, AevConst c, unsigned long long *__restrict__ Ffix,
                float *__restrict__ W_atom, Live n_cells) {
  extern __shared__ float4 lds4[];
  __shared__ int counter;
  if ((int)blockIdx.x >= n_cells.get()) return;  // the whole workgroup leaves together
  const int b = cell_start[blockIdx.x], e = cell_start[blockIdx.x + 1];
  if (b == e) return;  // the whole workgroup leaves together
  char *tail = (char *)lds4 + WPB * wave_lds_bytes<true>(cap);
  unsigned long long *hval = (unsigned long long *)tail;
  int *hkey = (int *)(tail + 24 * kBwdHash);
  for (int t = threadIdx.x; t < kBwdHash; t += WPB * kWave) {
    hkey[t] = -1;
    hval[3 * t] = hval[3 * t + 1] = hval[3 * t + 2] = 0ull;
  }
  if (threadIdx.x == 0) counter = 0;
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  WaveLds w = carve<true>((char *)lds4 + wave * wave_lds_bytes<true>(cap), cap);
  // a cell's centres and their neighbours belong to one system
  const int shift = fix_shift(sys[sys_of[cell_atoms[b]]]);
  const SinkHash sink{hkey, hval, Ffix, shift};
  for (int p = next_centre(&counter, lane); b + p < e; p = next_centre(&counter, lane))
    bwd_centre(cell_atoms[b + p], lane, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, c, W_atom, w,
               sink);
  __syncthreads();
  for (int t = threadIdx.x; t < kBwdHash; t += WPB * kWave) {
    const int j = hkey[t];
    if (j < 0) continue;
    unsigned long long *p = Ffix + 3 * (size_t)(j + shift);
    for (int q = 0; q < 3; ++q) {
      const unsigned long long v = hval[3 * t + q];
      if (v) atomicAdd(p + q, v);
    }
  }
}

// Waves per workgroup: the preference (1, 2 or 4) when its LDS fits in
// 64 KB, else one.  One is the default: each wave works on its own centre,
// and single-wave workgroups pack the compute units most freely (it was the
// fastest shape on most measured batches).
template <bool BWD>
static int waves_for_cap(int cap, int pref) {
  const size_t per = wave_lds_bytes<BWD>(cap);
  if ((pref == 1 || pref == 2 || pref == 4) && per * pref <= 64 * 1024) return pref;
  return 1;
}

template <bool BF16>
static void aev_fwd_t(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                      const int *nbr_cnt, int cap, const int *row_of_atom, void *G, int ldg,
                      unsigned long long *row_mask, const int *wave_atom, int *status, Live N, const AevConst &c,
                      int wpb_pref, hipStream_t st) {
  int wpb = waves_for_cap<false>(cap, wpb_pref);
  size_t lds = wave_lds_bytes<false>(cap) * wpb;
  unsigned grid = (unsigned)((N.v + wpb - 1) / wpb);
  if (wpb == 4)
    k_aev_fwd<4, BF16><<<grid, 4 * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg,
                                                     row_mask, wave_atom, status, N, c);
  else if (wpb == 2)
    k_aev_fwd<2, BF16><<<grid, 2 * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg,
                                                     row_mask, wave_atom, status, N, c);
  else
    k_aev_fwd<1, BF16><<<grid, kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg,
                                                 row_mask, wave_atom, status, N, c);
}

void launch_aev_fwd(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                    const int *nbr_cnt, int cap, const int *row_of_atom, void *G, bool g_bf16,
                    int ldg, Live N, const AevConst &c, unsigned long long *row_mask, const int *wave_atom,
                    int *status, int wpb_pref, hipStream_t st) {
  if (N.v <= 0) return;
  if (g_bf16)
    aev_fwd_t<true>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, row_mask, wave_atom, status, N, c,
                    wpb_pref, st);
  else
    aev_fwd_t<false>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, row_mask, wave_atom, status, N, c,
                     wpb_pref, st);
}

template <int WPB>
static void aev_bwd_launch(int form, size_t lds, unsigned grid, const AevBwdGroups &gp, const float4 *pos,
                           const int *sys_of, const SysDesc *sys, const int2 *nbr, const int *nbr_cnt, int cap,
                           const int *row_of_atom, const float *dG, int ldg, Live N, const AevConst &c,
                           unsigned long long *Ffix, float *W_atom, hipStream_t st) {
  if constexpr (WPB >= 4) {  // grouped forms run 4 to 10 waves per workgroup
    if (form == 1) {
      k_aev_bwd_sys<WPB><<<grid, WPB * kWave, lds, st>>>(gp.groups, pos, sys_of, sys, nbr, nbr_cnt, cap,
                                                         row_of_atom, dG, ldg, c, Ffix, W_atom,
                                                         Live(gp.n_groups, gp.live_groups));
      return;
    }
    if (form == 2) {
      k_aev_bwd_cells<WPB><<<grid, WPB * kWave, lds, st>>>(gp.cell_start, gp.cell_atoms, pos, sys_of, sys, nbr,
                                                           nbr_cnt, cap, row_of_atom, dG, ldg, c, Ffix, W_atom,
                                                           Live(gp.n_cells, gp.live_cells));
      return;
    }
  }
  if constexpr (WPB <= 4)
    k_aev_bwd<WPB><<<grid, WPB * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c,
                                                   Ffix, W_atom, gp.wave_atom);
}

// Chooses the form.  wpb_pref 0 (untuned), 1 or 2: one wave per centre,
// forces straight into Ffix by device atomics, one or two waves per
// workgroup (the fastest form measured on the ragged solutes and on the
// 100k-atom box).  4, 5, 6, 8 or 10: a grouped form when the call has one,
// with that many waves per workgroup (fewer when the LDS does not hold
// them): per system for a batch of small non-periodic systems (gp.groups),
// per cell on a grid of at least kBwdMinCells cells (fewer would leave
// compute units idle).  Without a grouped form: one wave per centre.
void launch_aev_bwd(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                    const int *nbr_cnt, int cap, const int *row_of_atom, const float *dG, int ldg,
                    Live N, const AevConst &c, unsigned long long *Ffix, float *W_atom, const AevBwdGroups &gp,
                    int wpb_pref, size_t max_lds, hipStream_t st) {
  if (N.v <= 0) return;
  const size_t per = wave_lds_bytes<true>(cap);
  int form = 0;
  size_t table = 0;
  if (wpb_pref >= 4) {
    if (gp.groups && gp.n_groups > 0) {
      form = 1;
      table = ((size_t)gp.max_sys_atoms * 24 + 15) / 16 * 16;
    } else if (gp.cell_start && gp.n_cells >= kBwdMinCells) {
      form = 2;
      table = (size_t)kBwdHash * 28;
    }
  }
  if (form) {
    // kBwdStaticLds: the kernels' static LDS (the centre counter) comes on
    // top of the dynamic allocation
    int wpb = (wpb_pref == 4 || wpb_pref == 5 || wpb_pref == 6 || wpb_pref == 8 || wpb_pref == 10) ? wpb_pref : 8;
    auto fits = [&](int w) { return per * w + table + kBwdStaticLds <= max_lds; };
    while (wpb >= 4 && !fits(wpb)) wpb = wpb == 10 ? 8 : wpb == 8 ? 6 : wpb - 1;
    if (wpb >= 4) {
      const size_t lds = per * wpb + table;
      const unsigned grid = (unsigned)(form == 1 ? gp.n_groups : gp.n_cells);
#define NNP_BWD_CASE(W)                                                                                     \
  case W:                                                                                                   \
    aev_bwd_launch<W>(form, lds, grid, gp, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, \
                      Ffix, W_atom, st);                                                                    \
    return;
      switch (wpb) {
        NNP_BWD_CASE(4)
        NNP_BWD_CASE(5)
        NNP_BWD_CASE(6)
        NNP_BWD_CASE(8)
        NNP_BWD_CASE(10)
        default: break;
      }
#undef NNP_BWD_CASE
    }
  }
  const int wpb = waves_for_cap<true>(cap, wpb_pref);
  const size_t lds = per * wpb;
  const unsigned grid = (unsigned)((N.v + wpb - 1) / wpb);
  if (wpb == 4)
    aev_bwd_launch<4>(0, lds, grid, gp, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, Ffix,
                      W_atom, st);
  else if (wpb == 2)
    aev_bwd_launch<2>(0, lds, grid, gp, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, Ffix,
                      W_atom, st);
  else
    aev_bwd_launch<1>(0, lds, grid, gp, pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, Ffix,
                      W_atom, st);
}

}  // namespace nnp
