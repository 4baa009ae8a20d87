// Element networks (section "Neural Network Potentials": one feed-forward
// network per element; the total energy is the sum of atomic energies,
// energy-decomposition equation) and the float64 per-system reductions.
//
// Dense layers are grouped GEMMs over species buckets: rows of one species
// are contiguous and padded to 128, so a 128-row tile always belongs to one
// network and every launch covers all species of one layer index.
//   C[rows, n_out] = A[rows, 0:K] . B[n_out, 0:K]^T  with a fused epilogue:
//     forward:  CELU(acc + bias)                    -> hidden activations
//     backward: acc * CELU'(layer input)            -> input gradient
//     output:   (C +=) acc * scale                  -> dE/dG
// MFMA: v_mfma_f32_32x32x2_f32 (float32 form) or v_mfma_f32_32x32x16_bf16
// (bfloat16 operands, float32 accumulate).  A workgroup of 4 waves computes a
// 128 x 64 tile; each wave a 32 x 64 strip as two 32x32 MFMA blocks that
// share the A fragment.
#include "internal.h"

namespace nnp {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTN = 64;

__device__ inline uint32_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ inline uint2 pack4_bf16(float4 v) {
  uint2 r;
  r.x = bf16_bits_rne(v.x) | (bf16_bits_rne(v.y) << 16);
  r.y = bf16_bits_rne(v.z) | (bf16_bits_rne(v.w) << 16);
  return r;
}

__device__ inline float celu(float z, float alpha) { return z > 0.f ? z : alpha * expm1f(z / alpha); }

// CELU'(z) from h = CELU(z): 1 for h > 0, else exp(z / alpha) = 1 + h / alpha.
__device__ inline float dcelu_from_h(float h, float alpha) { return h > 0.f ? 1.f : 1.f + h / alpha; }

template <int EPI, bool BF16>
__global__ void __launch_bounds__(256) k_gemm(GemmLaunch gl) {
  constexpr int TM = kTileM, TN = kTN;
  constexpr int TK = BF16 ? 64 : 32;
  constexpr int PADF = 1;   // float32 row padding (words)
  constexpr int PADH = 8;   // bf16 row padding (halves)
  constexpr int LDA = BF16 ? TK + PADH : TK + PADF;
  __shared__ __attribute__((aligned(16))) char smem[BF16 ? (TM + TN) * LDA * 2 : (TM + TN) * LDA * 4];

  const int r0 = blockIdx.x * TM;
  int s = -1;
  for (int q = 0; q < gl.n_groups; ++q)
    if (r0 >= gl.bucket_off[q] && r0 < gl.bucket_off[q + 1]) s = q;
  if (s < 0) return;
  const GemmGroup grp = gl.g[s];
  const int c0 = blockIdx.y * TN;
  if (c0 >= grp.n_out) return;
  const int K = grp.K;
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int l32 = lane & 31, hi = lane >> 5;

  floatx16 acc0 = {}, acc1 = {};
  const float *A = gl.A + (size_t)r0 * gl.lda;

  for (int k0 = 0; k0 < K; k0 += TK) {
    if (BF16) {
      uint16_t *As = (uint16_t *)smem;
      uint16_t *Bs = As + TM * LDA;
      // A: TM x TK floats -> bf16
#pragma unroll
      for (int q = 0; q < (TM * TK / 4) / 256; ++q) {
        int idx = q * 256 + tid;
        int row = idx / (TK / 4), c4 = idx % (TK / 4);
        int k = k0 + c4 * 4;
        float4 v = k < K ? *(const float4 *)(A + (size_t)row * gl.lda + k) : make_float4(0.f, 0.f, 0.f, 0.f);
        *(uint2 *)(As + row * LDA + c4 * 4) = pack4_bf16(v);
      }
      // B: TN x TK bf16, 8 per load
      const uint16_t *B = (const uint16_t *)grp.B;
#pragma unroll
      for (int q = 0; q < (TN * TK / 8) / 256; ++q) {
        int idx = q * 256 + tid;
        int row = idx / (TK / 8), c8 = idx % (TK / 8);
        int k = k0 + c8 * 8, col = c0 + row;
        uint4 v = (k < K && col < grp.n_out) ? *(const uint4 *)(B + (size_t)col * K + k)
                                             : make_uint4(0u, 0u, 0u, 0u);
        *(uint4 *)(Bs + row * LDA + c8 * 8) = v;
      }
    } else {
      float *As = (float *)smem;
      float *Bs = As + TM * LDA;
#pragma unroll
      for (int q = 0; q < (TM * TK / 4) / 256; ++q) {
        int idx = q * 256 + tid;
        int row = idx / (TK / 4), c4 = idx % (TK / 4);
        int k = k0 + c4 * 4;
        float4 v = k < K ? *(const float4 *)(A + (size_t)row * gl.lda + k) : make_float4(0.f, 0.f, 0.f, 0.f);
        float *d = As + row * LDA + c4 * 4;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      }
      const float *B = (const float *)grp.B;
#pragma unroll
      for (int q = 0; q < (TN * TK / 4) / 256; ++q) {
        int idx = q * 256 + tid;
        int row = idx / (TK / 4), c4 = idx % (TK / 4);
        int k = k0 + c4 * 4, col = c0 + row;
        float4 v = (k < K && col < grp.n_out) ? *(const float4 *)(B + (size_t)col * K + k)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
        float *d = Bs + row * LDA + c4 * 4;
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      }
    }
    __syncthreads();
    if (BF16) {
      const uint16_t *As = (const uint16_t *)smem;
      const uint16_t *Bs = As + TM * LDA;
#pragma unroll
      for (int kk = 0; kk < TK; kk += 16) {
        bf16x8 a = __builtin_bit_cast(bf16x8, *(const uint4 *)(As + (wave * 32 + l32) * LDA + kk + 8 * hi));
        bf16x8 b0 = __builtin_bit_cast(bf16x8, *(const uint4 *)(Bs + l32 * LDA + kk + 8 * hi));
        bf16x8 b1 = __builtin_bit_cast(bf16x8, *(const uint4 *)(Bs + (32 + l32) * LDA + kk + 8 * hi));
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
      }
    } else {
      const float *As = (const float *)smem;
      const float *Bs = As + TM * LDA;
#pragma unroll
      for (int kk = 0; kk < TK; kk += 2) {
        float a = As[(wave * 32 + l32) * LDA + kk + hi];
        float b0 = Bs[l32 * LDA + kk + hi];
        float b1 = Bs[(32 + l32) * LDA + kk + hi];
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // D[row][col]: col = lane % 32, row = 8 (i / 4) + 4 (lane / 32) + i % 4
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int col = c0 + blk * 32 + l32;
    if (col >= grp.n_out) continue;
    float bias = 0.f;
    if (EPI == kEpiFwd) bias = grp.bias[col];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = r0 + wave * 32 + 8 * (i / 4) + 4 * hi + (i % 4);
      float v = blk == 0 ? acc0[i] : acc1[i];
      float *out = gl.C + (size_t)row * gl.ldc + col;
      if (EPI == kEpiFwd) {
        *out = celu(v + bias, gl.alpha);
      } else if (EPI == kEpiBwd) {
        const float h = gl.H[(size_t)row * gl.ldh + col];
        *out = v * dcelu_from_h(h, gl.alpha) * gl.scale;
      } else {
        v *= gl.scale;
        *out = gl.accumulate ? *out + v : v;
      }
    }
  }
}

void launch_gemm(int epi, bool bf16, const GemmLaunch &gl, int row_tiles, int max_n_out,
                 hipStream_t st) {
  if (row_tiles <= 0) return;
  dim3 grid(row_tiles, (max_n_out + kTN - 1) / kTN);
  if (bf16) {
    if (epi == kEpiFwd) k_gemm<kEpiFwd, true><<<grid, 256, 0, st>>>(gl);
    else if (epi == kEpiBwd) k_gemm<kEpiBwd, true><<<grid, 256, 0, st>>>(gl);
    else k_gemm<kEpiOut, true><<<grid, 256, 0, st>>>(gl);
  } else {
    if (epi == kEpiFwd) k_gemm<kEpiFwd, false><<<grid, 256, 0, st>>>(gl);
    else if (epi == kEpiBwd) k_gemm<kEpiBwd, false><<<grid, 256, 0, st>>>(gl);
    else k_gemm<kEpiOut, false><<<grid, 256, 0, st>>>(gl);
  }
}

// Output layer (one unit): E_row = w . h + b, and dE/dh = w * CELU'(h) (or
// w itself when the network has no hidden layer), both scaled by 1/M for an
// ensemble of M networks.  One wave per row.
__global__ void __launch_bounds__(256) k_energy(EnergyLaunch el, int rows) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int row = blockIdx.x * 4 + wave;
  if (row >= rows) return;
  int s = -1;
  for (int q = 0; q < el.n_groups; ++q)
    if (row >= el.bucket_off[q] && row < el.bucket_off[q + 1]) s = q;
  if (s < 0) return;
  const int atom = el.perm[row];
  if (atom < 0) return;
  const int K = el.K[s];
  const float *w = el.w[s];
  const float *h = el.Hin + (size_t)row * el.ldh;
  float *go = el.Gout + (size_t)row * el.ldg;
  float e = 0.f;
  for (int k = lane; k < K; k += kWave) {
    const float hv = h[k], wv = w[k];
    e += hv * wv;
    if (el.want_grad) {
      float gk = (el.hidden ? wv * dcelu_from_h(hv, el.alpha) : wv) * el.inv_m;
      go[k] = el.accumulate_grad ? go[k] + gk : gk;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) e += __shfl_xor(e, off);
  if (lane == 0) {
    const float val = (e + el.b[s][0]) * el.inv_m;
    el.e_atom[atom] = el.first ? val : el.e_atom[atom] + val;
  }
}

void launch_energy(const EnergyLaunch &el, int rows, hipStream_t st) {
  if (rows <= 0) return;
  k_energy<<<(rows + 3) / 4, 256, 0, st>>>(el, rows);
}

// Per-system totals in float64: energies (sum of atomic energies) and the
// virial (sum of per-centre virials).  Deterministic two-level sum: fixed
// chunks of at most 4096 atoms, then the chunks of each system in order.
constexpr int kChunk = 4096;

__global__ void __launch_bounds__(256)
k_reduce_partial(const float *__restrict__ e_atom, const float *__restrict__ W_atom,
                 const SysDesc *__restrict__ sys, const int *__restrict__ chunk_sys,
                 const int *__restrict__ chunk_begin, double *__restrict__ partial) {
  __shared__ double red[10][256 / kWave];
  const int ch = blockIdx.x;
  const SysDesc &d = sys[chunk_sys[ch]];
  const int b = chunk_begin[ch];
  const int e = min(b + kChunk, d.atom_off + d.n);
  double acc[10];
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
    acc[0] += (double)e_atom[i];
    if (W_atom)
      for (int q = 0; q < 9; ++q) acc[1 + q] += (double)W_atom[(size_t)9 * i + q];
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (int q = 0; q < 10; ++q) {
    double v = acc[q];
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    double v = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) v += red[threadIdx.x][w];
    partial[(size_t)10 * ch + threadIdx.x] = v;
  }
}

__global__ void k_reduce_final(const double *__restrict__ partial, const int *__restrict__ sys_chunk_off,
                               int n_sys, double *__restrict__ energy, double *__restrict__ virial) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  double acc[10];
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int ch = sys_chunk_off[s]; ch < sys_chunk_off[s + 1]; ++ch)
    for (int q = 0; q < 10; ++q) acc[q] += partial[(size_t)10 * ch + q];
  energy[s] = acc[0];
  if (virial)
    for (int q = 0; q < 9; ++q) virial[(size_t)9 * s + q] = acc[1 + q];
}

void launch_reduce(const float *e_atom, const float *W_atom, const SysDesc *sys, int n_sys,
                   const int *chunk_sys, const int *chunk_begin, int n_chunks,
                   const int *sys_chunk_off, double *partial, double *energy, double *virial,
                   hipStream_t st) {
  if (n_chunks > 0)
    k_reduce_partial<<<n_chunks, 256, 0, st>>>(e_atom, W_atom, sys, chunk_sys, chunk_begin, partial);
  if (n_sys > 0)
    k_reduce_final<<<(n_sys + 127) / 128, 128, 0, st>>>(partial, sys_chunk_off, n_sys, energy, virial);
}

}  // namespace nnp
