// Atomic environment vectors and their gradient (section "ANI models":
// cosine cutoff, radial and angular symmetry functions).
//
// One wavefront per centre atom.  The centre's neighbour entries are
// re-derived from the packed atom records, sorted by neighbour species into
// LDS with wave ballots, and then
//   radial:  lanes = 16 radial shifts x 4 neighbour slots, one species block
//            at a time, reduced across the 4 slots with lane shuffles;
//   angular: lanes = 8 angle shifts x 8 neighbour pairs, one species-pair
//            block at a time.  Each lane evaluates the cosine power for its
//            own angle shift and one of the 4 radial Gaussians, which the
//            8 lanes of a pair then exchange; the 4 radial-shift accumulators
//            are reduced across the 8 pairs at the end of the block.
// The backward kernel walks the same blocks with dE/dG, accumulates
// dE/dd per neighbour entry in LDS and scatters forces with float atomics.
#include "internal.h"

namespace nnp {

constexpr float kPi = 3.14159265358979323846f;

__device__ inline unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
}

__device__ inline float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

// Pair (j < k) of the same-species block with n entries from its rank t in
// row-major order over the strict upper triangle.
__device__ inline void unrank_upper(int t, int n, int &j, int &k) {
  float fn = (float)(2 * n - 1);
  int jj = (int)((fn - sqrtf(fmaxf(fn * fn - 8.0f * (float)t, 0.f))) * 0.5f);
  jj = max(0, min(jj, n - 2));
  auto start = [n](int r) { return r * (2 * n - r - 1) / 2; };
  while (jj > 0 && start(jj) > t) --jj;
  while (jj < n - 2 && start(jj + 1) <= t) ++jj;
  j = jj;
  k = t - start(jj) + jj + 1;
}

// Wave-uniform per-species counts and offsets of the sorted lists.
struct Lists {
  int cR[kMaxSpecies], oR[kMaxSpecies];
  int cA[kMaxSpecies], oA[kMaxSpecies];
};

// Neighbour vector d = r_j + image * L - r_i of entry e of centre i.
__device__ inline float4 entry_vec(const float4 &pi, const float4 &pj, int code, const float L[3]) {
  int ix, iy, iz;
  unpack_image(code, ix, iy, iz);
  float dx = (pj.x - pi.x) + (float)ix * L[0];
  float dy = (pj.y - pi.y) + (float)iy * L[1];
  float dz = (pj.z - pi.z) + (float)iz * L[2];
  return make_float4(dx, dy, dz, sqrtf(dx * dx + dy * dy + dz * dz));
}

// LDS layout of one wave's lists (cap entries each).
struct WaveLds {
  float4 *rD;   // radial: d vector and R
  float *rFc;   // radial: fc_rad(R)
  float *rDfc;  // radial: fc_rad'(R)         (backward)
  int *rJ;      // radial: neighbour index     (backward)
  float *rG;    // radial: dE/dd accumulators  (backward, 3 per entry)
  int *aIdx;    // angular: position in the radial arrays
  float *aFc;   // angular: fc_ang(R)
  float *aDfc;  // angular: fc_ang'(R)         (backward)
};

template <bool BWD>
__host__ __device__ inline size_t wave_lds_bytes(int cap) {
  return (size_t)cap * (BWD ? 16 + 4 + 4 + 4 + 12 + 4 + 4 + 4 : 16 + 4 + 4 + 4);
}

template <bool BWD>
__device__ inline WaveLds carve(char *base, int cap) {
  WaveLds w{};
  w.rD = (float4 *)base;
  char *p = base + (size_t)cap * 16;
  w.rFc = (float *)p; p += (size_t)cap * 4;
  w.aIdx = (int *)p; p += (size_t)cap * 4;
  w.aFc = (float *)p; p += (size_t)cap * 4;
  if (BWD) {
    w.rDfc = (float *)p; p += (size_t)cap * 4;
    w.rJ = (int *)p; p += (size_t)cap * 4;
    w.rG = (float *)p; p += (size_t)cap * 12;
    w.aDfc = (float *)p; p += (size_t)cap * 4;
  }
  return w;
}

// Builds the species-sorted radial list (R < rc_r) and angular list
// (R < rc_a, a subset) of centre i in LDS.  Two passes over the entries:
// per-species counts by ballot, then placement.
template <bool BWD>
__device__ inline void fill_lists(int lane, int n, const int2 *__restrict__ ent,
                                  const float4 *__restrict__ pos, const float4 &pi,
                                  const float L[3], const AevConst &c, WaveLds &w, Lists &ls) {
  const int S = c.S;
  for (int s = 0; s < kMaxSpecies; ++s) { ls.cR[s] = 0; ls.cA[s] = 0; }
  for (int b = 0; b < n; b += kWave) {
    int e = b + lane;
    bool v = e < n;
    int sj = -1;
    float R = 1e30f;
    if (v) {
      int2 en = ent[e];
      float4 pj = pos[en.x];
      R = entry_vec(pi, pj, en.y, L).w;
      sj = __float_as_int(pj.w);
    }
    bool inR = v && R < c.rc_r, inA = v && R < c.rc_a;
    for (int s = 0; s < S; ++s) {
      ls.cR[s] += __popcll(__ballot(inR && sj == s));
      ls.cA[s] += __popcll(__ballot(inA && sj == s));
    }
  }
  int oR = 0, oA = 0;
  for (int s = 0; s < S; ++s) {
    ls.oR[s] = oR; oR += ls.cR[s];
    ls.oA[s] = oA; oA += ls.cA[s];
  }
  int pR[kMaxSpecies], pA[kMaxSpecies];
  for (int s = 0; s < S; ++s) { pR[s] = ls.oR[s]; pA[s] = ls.oA[s]; }
  const float kr = kPi / c.rc_r, ka = kPi / c.rc_a;
  for (int b = 0; b < n; b += kWave) {
    int e = b + lane;
    bool v = e < n;
    int sj = -1, j = 0;
    float4 d = make_float4(0.f, 0.f, 0.f, 1e30f);
    if (v) {
      int2 en = ent[e];
      float4 pj = pos[en.x];
      d = entry_vec(pi, pj, en.y, L);
      sj = __float_as_int(pj.w);
      j = en.x;
    }
    bool inR = v && d.w < c.rc_r, inA = v && d.w < c.rc_a;
    for (int s = 0; s < S; ++s) {
      unsigned long long mR = __ballot(inR && sj == s);
      unsigned long long mA = __ballot(inA && sj == s);
      int q = pR[s] + (int)lanes_below(mR);
      if (inR && sj == s) {
        float sn, cs;
        __sincosf(kr * d.w, &sn, &cs);
        w.rD[q] = d;
        w.rFc[q] = 0.5f * cs + 0.5f;
        if (BWD) {
          w.rDfc[q] = -0.5f * kr * sn;
          w.rJ[q] = j;
          w.rG[3 * q] = 0.f; w.rG[3 * q + 1] = 0.f; w.rG[3 * q + 2] = 0.f;
        }
      }
      if (inA && sj == s) {
        int qa = pA[s] + (int)lanes_below(mA);
        float sn, cs;
        __sincosf(ka * d.w, &sn, &cs);
        w.aIdx[qa] = q;
        w.aFc[qa] = 0.5f * cs + 0.5f;
        if (BWD) w.aDfc[qa] = -0.5f * ka * sn;
      }
      pR[s] += __popcll(mR);
      pA[s] += __popcll(mA);
    }
  }
}

template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_aev_fwd(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
          const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
          const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
          float *__restrict__ G, int ldg, int N, AevConst c) {
  extern __shared__ float4 lds4[];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int i = blockIdx.x * WPB + wave;
  const bool live = i < N;
  WaveLds w = carve<false>((char *)lds4 + wave * wave_lds_bytes<false>(cap), cap);
  Lists ls;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  float L[3] = {0.f, 0.f, 0.f};
  int n = 0;
  if (live) {
    n = min(nbr_cnt[i], cap);
    pi = pos[i];
    const SysDesc &d = sys[sys_of[i]];
    L[0] = d.L[0]; L[1] = d.L[1]; L[2] = d.L[2];
  }
  fill_lists<false>(lane, n, nbr + (size_t)(live ? i : 0) * cap, pos, pi, L, c, w, ls);
  __syncthreads();
  if (!live) return;
  float *Grow = G + (size_t)row_of_atom[i] * ldg;

  // radial: G[16 s + m] = scale * sum_j exp(-eta (R - Rs_m)^2) fc(R)
  {
    const int m = lane & 15, slot = lane >> 4;
    const float shf = c.shf_r[m];
    for (int s = 0; s < c.S; ++s) {
      float acc = 0.f;
      const int o = ls.oR[s];
      for (int e = slot; e < ls.cR[s]; e += 4) {
        float R = w.rD[o + e].w;
        float t = R - shf;
        acc += fast_exp(-c.eta_r * t * t) * w.rFc[o + e];
      }
      acc += __shfl_xor(acc, 16);
      acc += __shfl_xor(acc, 32);
      if (slot == 0) Grow[s * kNShfRad + m] = acc * c.scale;
    }
  }

  // angular
  {
    const int a = lane & 7, t0 = lane >> 3, grp = lane & ~7;
    const float cza = c.cz[a], sza = c.sz[a], shf_own = c.shf_a[a & 3];
    const float pre = 1.0f - c.zeta;
    int p = 0;
    for (int sa = 0; sa < c.S; ++sa) {
      for (int sb = sa; sb < c.S; ++sb, ++p) {
        const int na = ls.cA[sa], nb = ls.cA[sb];
        const int T = sa == sb ? na * (na - 1) / 2 : na * nb;
        float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;
        for (int base = 0; base < T; base += 8) {
          const int t = base + t0;
          const bool valid = t < T;
          const int tt = valid ? t : T - 1;
          int j, k;
          if (sa == sb) unrank_upper(tt, na, j, k);
          else { j = tt / nb; k = tt - j * nb; }
          const int qj = ls.oA[sa] + j, qk = ls.oA[sb] + k;
          const float4 dj = w.rD[w.aIdx[qj]], dk = w.rD[w.aIdx[qk]];
          const float fj = w.aFc[qj], fk = w.aFc[qk];
          const float dot = dj.x * dk.x + dj.y * dk.y + dj.z * dk.z;
          const float cx = dj.y * dk.z - dj.z * dk.y;
          const float cy = dj.z * dk.x - dj.x * dk.z;
          const float cz = dj.x * dk.y - dj.y * dk.x;
          const float cr = sqrtf(cx * cx + cy * cy + cz * cz);
          const float inv = 1.0f / (dj.w * dk.w);
          const float cc = (dot * cza + cr * sza) * inv;  // cos(theta - theta_s)
          const float x = fmaxf(1.0f + cc, 0.f);
          const float f1 = fast_exp2(c.zeta * fast_log2(x) + pre);
          const float u = 0.5f * (dj.w + dk.w) - shf_own;
          const float f2 = fast_exp(-c.eta_a * u * u);
          const float f20 = __shfl(f2, grp | 0), f21 = __shfl(f2, grp | 1);
          const float f22 = __shfl(f2, grp | 2), f23 = __shfl(f2, grp | 3);
          const float v = valid ? f1 * fj * fk : 0.f;
          acc0 += v * f20; acc1 += v * f21; acc2 += v * f22; acc3 += v * f23;
        }
        for (int off = 8; off < kWave; off <<= 1) {
          acc0 += __shfl_xor(acc0, off);
          acc1 += __shfl_xor(acc1, off);
          acc2 += __shfl_xor(acc2, off);
          acc3 += __shfl_xor(acc3, off);
        }
        if (t0 == 0) {
          float *o = Grow + c.rad_len + p * kAngBlock + a;
          o[0] = acc0; o[kNShfZ] = acc1; o[2 * kNShfZ] = acc2; o[3 * kNShfZ] = acc3;
        }
      }
    }
  }
}

template <int WPB>
__global__ void __launch_bounds__(WPB * kWave)
k_aev_bwd(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
          const SysDesc *__restrict__ sys, const int2 *__restrict__ nbr,
          const int *__restrict__ nbr_cnt, int cap, const int *__restrict__ row_of_atom,
          const float *__restrict__ dG, int ldg, int N, AevConst c, float *__restrict__ F,
          float *__restrict__ W_atom) {
  extern __shared__ float4 lds4[];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int i = blockIdx.x * WPB + wave;
  const bool live = i < N;
  WaveLds w = carve<true>((char *)lds4 + wave * wave_lds_bytes<true>(cap), cap);
  Lists ls;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  float L[3] = {0.f, 0.f, 0.f};
  int n = 0;
  if (live) {
    n = min(nbr_cnt[i], cap);
    pi = pos[i];
    const SysDesc &d = sys[sys_of[i]];
    L[0] = d.L[0]; L[1] = d.L[1]; L[2] = d.L[2];
  }
  fill_lists<true>(lane, n, nbr + (size_t)(live ? i : 0) * cap, pos, pi, L, c, w, ls);
  __syncthreads();
  if (!live) return;
  const float *g = dG + (size_t)row_of_atom[i] * ldg;

  // radial: dE/dR = scale * sum_m g_m d/dR[exp(-eta (R - Rs_m)^2) fc(R)]
  {
    const int m = lane & 15, slot = lane >> 4;
    const float shf = c.shf_r[m];
    for (int s = 0; s < c.S; ++s) {
      const float gm = g[s * kNShfRad + m] * c.scale;
      const int o = ls.oR[s];
      for (int e = slot; e < ls.cR[s]; e += 4) {
        const float4 d = w.rD[o + e];
        const float t = d.w - shf;
        const float ex = fast_exp(-c.eta_r * t * t);
        float term = gm * ex * (-2.0f * c.eta_r * t * w.rFc[o + e] + w.rDfc[o + e]);
        term += __shfl_xor(term, 1);
        term += __shfl_xor(term, 2);
        term += __shfl_xor(term, 4);
        term += __shfl_xor(term, 8);
        if (m == 0) {
          const float q = term / d.w;
          float *gg = w.rG + 3 * (o + e);
          gg[0] = q * d.x; gg[1] = q * d.y; gg[2] = q * d.z;
        }
      }
    }
  }

  // angular
  {
    const int a = lane & 7, t0 = lane >> 3, grp = lane & ~7;
    const float cza = c.cz[a], sza = c.sz[a], shf_own = c.shf_a[a & 3];
    const float pre = 1.0f - c.zeta;
    const float m2eta = -2.0f * c.eta_a;
    int p = 0;
    for (int sa = 0; sa < c.S; ++sa) {
      for (int sb = sa; sb < c.S; ++sb, ++p) {
        const int na = ls.cA[sa], nb = ls.cA[sb];
        const int T = sa == sb ? na * (na - 1) / 2 : na * nb;
        if (T == 0) continue;
        const float *gp = g + c.rad_len + p * kAngBlock + a;
        const float g0 = gp[0], g1 = gp[kNShfZ], g2 = gp[2 * kNShfZ], g3 = gp[3 * kNShfZ];
        for (int base = 0; base < T; base += 8) {
          const int t = base + t0;
          const bool valid = t < T;
          const int tt = valid ? t : T - 1;
          int j, k;
          if (sa == sb) unrank_upper(tt, na, j, k);
          else { j = tt / nb; k = tt - j * nb; }
          const int aj = ls.oA[sa] + j, ak = ls.oA[sb] + k;
          const int qj = w.aIdx[aj], qk = w.aIdx[ak];
          const float4 dj = w.rD[qj], dk = w.rD[qk];
          const float fj = w.aFc[aj], fk = w.aFc[ak];
          const float dfj = w.aDfc[aj], dfk = w.aDfc[ak];
          const float dot = dj.x * dk.x + dj.y * dk.y + dj.z * dk.z;
          const float cx = dj.y * dk.z - dj.z * dk.y;
          const float cy = dj.z * dk.x - dj.x * dk.z;
          const float cz = dj.x * dk.y - dj.y * dk.x;
          const float cr = sqrtf(cx * cx + cy * cy + cz * cz);
          const float RR = dj.w * dk.w;
          const float invRR = 1.0f / RR;
          const float cosv = dot * invRR, sinv = cr * invRR;
          const float x = fmaxf(1.0f + cosv * cza + sinv * sza, 0.f);
          // p1 = 2^(1-zeta) x^(zeta-1); f1 = p1 x; df1/dx = zeta p1
          const float p1 = fast_exp2((c.zeta - 1.0f) * fast_log2(x) + pre);
          const float f1 = p1 * x, df1 = c.zeta * p1;
          const float Rbar = 0.5f * (dj.w + dk.w);
          const float u = Rbar - shf_own;
          const float f2 = fast_exp(-c.eta_a * u * u);
          const float f20 = __shfl(f2, grp | 0), f21 = __shfl(f2, grp | 1);
          const float f22 = __shfl(f2, grp | 2), f23 = __shfl(f2, grp | 3);
          const float A = g0 * f20 + g1 * f21 + g2 * f22 + g3 * f23;
          const float B = m2eta * (g0 * (Rbar - c.shf_a[0]) * f20 + g1 * (Rbar - c.shf_a[1]) * f21 +
                                   g2 * (Rbar - c.shf_a[2]) * f22 + g3 * (Rbar - c.shf_a[3]) * f23);
          const float fcc = fj * fk;
          const float dVdc = valid ? df1 * A * fcc : 0.f;
          float dcos = dVdc * cza, dsin = dVdc * sza;
          float dRj = valid ? f1 * (0.5f * B * fcc + A * dfj * fk) : 0.f;
          float dRk = valid ? f1 * (0.5f * B * fcc + A * fj * dfk) : 0.f;
          for (int off = 1; off < 8; off <<= 1) {
            dcos += __shfl_xor(dcos, off);
            dsin += __shfl_xor(dsin, off);
            dRj += __shfl_xor(dRj, off);
            dRk += __shfl_xor(dRk, off);
          }
          // lanes 0-2 of the pair own dE/dd_j (x,y,z), lanes 3-5 own dE/dd_k
          if (valid && a < 6) {
            const bool isj = a < 3;
            const int comp = isj ? a : a - 3;
            const float4 da = isj ? dj : dk, db = isj ? dk : dj;
            const float Ra = da.w, Rb = db.w;
            const float dac = comp == 0 ? da.x : (comp == 1 ? da.y : da.z);
            const float dbc = comp == 0 ? db.x : (comp == 1 ? db.y : db.z);
            const float invRa2 = 1.0f / (Ra * Ra);
            const float inv_cr = cr > 1e-12f * RR ? 1.0f / cr : 0.f;
            const float dcos_d = dbc * invRR - cosv * dac * invRa2;
            const float dsin_d = inv_cr != 0.f
                                     ? (Rb * Rb * dac - dot * dbc) * inv_cr * invRR - sinv * dac * invRa2
                                     : 0.f;
            const float val = dcos * dcos_d + dsin * dsin_d + (isj ? dRj : dRk) * dac / Ra;
            atomicAdd(&w.rG[3 * (isj ? qj : qk) + comp], val);
          }
        }
      }
    }
  }

  // scatter: F_i += dE/dd, F_j -= dE/dd, per-centre virial -sum d (x) dE/dd
  {
    int nR = 0;
    for (int s = 0; s < c.S; ++s) nR += ls.cR[s];
    float fi0 = 0.f, fi1 = 0.f, fi2 = 0.f;
    float vir[9];
    for (int q = 0; q < 9; ++q) vir[q] = 0.f;
    for (int e = lane; e < nR; e += kWave) {
      const float4 d = w.rD[e];
      const float gx = w.rG[3 * e], gy = w.rG[3 * e + 1], gz = w.rG[3 * e + 2];
      const int j = w.rJ[e];
      fi0 += gx; fi1 += gy; fi2 += gz;
      atomicAdd(&F[3 * j], -gx);
      atomicAdd(&F[3 * j + 1], -gy);
      atomicAdd(&F[3 * j + 2], -gz);
      vir[0] -= d.x * gx; vir[1] -= d.x * gy; vir[2] -= d.x * gz;
      vir[3] -= d.y * gx; vir[4] -= d.y * gy; vir[5] -= d.y * gz;
      vir[6] -= d.z * gx; vir[7] -= d.z * gy; vir[8] -= d.z * gz;
    }
    for (int off = 32; off >= 1; off >>= 1) {
      fi0 += __shfl_xor(fi0, off);
      fi1 += __shfl_xor(fi1, off);
      fi2 += __shfl_xor(fi2, off);
      for (int q = 0; q < 9; ++q) vir[q] += __shfl_xor(vir[q], off);
    }
    if (lane == 0) {
      atomicAdd(&F[3 * i], fi0);
      atomicAdd(&F[3 * i + 1], fi1);
      atomicAdd(&F[3 * i + 2], fi2);
    }
    if (lane < 9) {
      float v = vir[0];
      for (int q = 1; q < 9; ++q) v = lane == q ? vir[q] : v;
      W_atom[(size_t)9 * i + lane] = v;
    }
  }
}

template <bool BWD>
static int waves_for_cap(int cap) {
  size_t per = wave_lds_bytes<BWD>(cap);
  if (per * 4 <= 64 * 1024) return 4;
  if (per * 2 <= 64 * 1024) return 2;
  return 1;
}

void launch_aev_fwd(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                    const int *nbr_cnt, int cap, const int *row_of_atom, float *G, int ldg, int N,
                    const AevConst &c, hipStream_t st) {
  if (N <= 0) return;
  int wpb = waves_for_cap<false>(cap);
  size_t lds = wave_lds_bytes<false>(cap) * wpb;
  unsigned grid = (unsigned)((N + wpb - 1) / wpb);
  if (wpb == 4)
    k_aev_fwd<4><<<grid, 4 * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, N, c);
  else if (wpb == 2)
    k_aev_fwd<2><<<grid, 2 * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, N, c);
  else
    k_aev_fwd<1><<<grid, kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, G, ldg, N, c);
}

void launch_aev_bwd(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                    const int *nbr_cnt, int cap, const int *row_of_atom, const float *dG, int ldg,
                    int N, const AevConst &c, float *F, float *W_atom, hipStream_t st) {
  if (N <= 0) return;
  int wpb = waves_for_cap<true>(cap);
  size_t lds = wave_lds_bytes<true>(cap) * wpb;
  unsigned grid = (unsigned)((N + wpb - 1) / wpb);
  if (wpb == 4)
    k_aev_bwd<4><<<grid, 4 * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, F, W_atom);
  else if (wpb == 2)
    k_aev_bwd<2><<<grid, 2 * kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, F, W_atom);
  else
    k_aev_bwd<1><<<grid, kWave, lds, st>>>(pos, sys_of, sys, nbr, nbr_cnt, cap, row_of_atom, dG, ldg, N, c, F, W_atom);
}

}  // namespace nnp
