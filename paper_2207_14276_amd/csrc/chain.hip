// Fused hidden-layer chain of the element networks (section "Neural Network
// Potentials": one feed-forward network per element, atomic energies summed).
//
// After the first dense layer (a large GEMM over the AEV), the remaining
// layers of a network are narrow (<= 256 wide): run as separate GEMMs their
// activations make several round trips through HBM.  Here one workgroup
// takes 32 rows of one species bucket for one ensemble member and runs the
// rest of the network on chip (or 64 rows, RT = 2, when the LDS allows: each
// weight fragment loaded from L2 then feeds twice as many MFMAs, and weight
// traffic from L2 is what bounds this kernel):
//   forward   h_l = CELU(h_{l-1} W_l^T + b_l) for the hidden layers l >= 1,
//             E = h_last . w_out + b_out, d_last = w_out * CELU'(h_last) / M;
//   backward  d_{l-1} = (d_l W_l) * CELU'(h_{l-1}) down to d_0,
// keeping every h_l / d_l tile in LDS (bfloat16, rows padded by 8 elements)
// and writing only d_0 (the input gradient the AEV-gradient GEMM needs) and
// the member's energy per row.  The products use v_mfma_f32_16x16x32_bf16:
// with W waves per workgroup (4 or 8, a tuned launch shape) each wave owns
// every W-th 16-column block of a layer's output; it reads the A fragments
// of a K step from LDS once for all its blocks and loads the next step's B
// fragments (weights, L2-resident) during the current MFMAs.  Activations
// are rounded to bfloat16 exactly where the unfused path stores them.
#include "internal.h"

namespace nnp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (one hardware conversion)
__device__ inline uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// four floats -> four bfloat16 (round to nearest even) in 8 bytes, first value lowest
typedef __bf16 bf16x2_c __attribute__((ext_vector_type(2)));
typedef float floatx2_c __attribute__((ext_vector_type(2)));
__device__ inline uint2 pack4_bf16(float a, float b, float c, float d) {
  uint2 r;
  r.x = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2_c){a, b}, bf16x2_c));
  r.y = __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2_c){c, d}, bf16x2_c));
  return r;
}
// CELU with the hardware exp2 (about 1 ulp; the result is rounded to
// bfloat16 next), k_exp = log2(e) / alpha; CELU' from h = CELU(z) with
// inv_alpha = 1 / alpha.
__device__ inline float celu_f(float z, float alpha, float k_exp) {
  return z > 0.f ? z : alpha * (__builtin_amdgcn_exp2f(z * k_exp) - 1.f);
}
__device__ inline float dcelu_h(float h, float inv_alpha) { return h > 0.f ? 1.f : 1.f + h * inv_alpha; }

// Sum over aligned groups of 8 lanes (DPP), result in every lane of the group.
__device__ inline float sum8_dpp(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
  return v;
}

// C[32 RT x N] = A[32 RT x K] (LDS, bfloat16, row stride lda) . B^T with
// B[N][K] (global, bfloat16, row stride ldb); K a multiple of 32 (<= 256), N
// of 16.  Each product is formed transposed (weights as the MFMA's first
// operand), so that a lane ends with four consecutive columns of one row:
// for every 16-column block owned by this wave, epi(cb, acc) gets, in
// acc[h][j], row 16 h + l % 16 and column 16 cb + 4 (l / 16) + j (j = 0..3)
// of each of the 2 RT sixteen-row groups h; the epilogues then move four
// bfloat16 values (8 bytes) per LDS access.
template <int W, int RT, class Epi>
__device__ inline void chain_gemm(const uint16_t *A, int lda, int K, const uint16_t *__restrict__ B, int ldb,
                                  int N, int wave, int lane, Epi &&epi) {
  constexpr int QM = 16 / W;                      // blocks per wave at N = 256
  constexpr int HR = 2 * RT;                      // sixteen-row groups
  const int l16 = lane & 15, kq = lane >> 4;
  const int nkb = K / 32, ncb = N / 16;
  // this wave's blocks: wave + W q, q < nq (N <= 256: at most 16 / W).
  // K-step outer, blocks inner: the A fragments of a K step are read from
  // LDS once for all of the wave's blocks, and the next step's B fragments
  // are loaded while the current step's MFMAs run.
  const int nq = ncb > wave ? (ncb - wave + W - 1) / W : 0;
  if (nq == 0) return;
  floatx4_t acc[QM][HR];
#pragma unroll
  for (int q = 0; q < QM; ++q)
#pragma unroll
    for (int h = 0; h < HR; ++h) acc[q][h] = floatx4_t{0.f, 0.f, 0.f, 0.f};
  const uint16_t *bp = B + (size_t)(wave * 16 + l16) * ldb + 8 * kq;
  const size_t bstep = (size_t)16 * W * ldb;      // W blocks of 16 rows
  // B fragments of K steps kb (bc), kb + 1 (bn) and kb + 2 (bnn): the loads
  // (L2 hits) are issued two steps ahead of their MFMAs
  uint4 bc[QM], bn[QM], bnn[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q)
    if (q < nq) {
      bc[q] = *(const uint4 *)(bp + q * bstep);
      if (nkb > 1) bn[q] = *(const uint4 *)(bp + q * bstep + 32);
    }
  for (int kb = 0; kb < nkb; ++kb) {
    if (kb + 2 < nkb) {
#pragma unroll
      for (int q = 0; q < QM; ++q)
        if (q < nq) bnn[q] = *(const uint4 *)(bp + q * bstep + (kb + 2) * 32);
    }
    bf16x8_t a[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h)
      a[h] = __builtin_bit_cast(bf16x8_t, *(const uint4 *)(A + (16 * h + l16) * lda + kb * 32 + 8 * kq));
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      if (q < nq) {
        const bf16x8_t b = __builtin_bit_cast(bf16x8_t, bc[q]);
#pragma unroll
        for (int h = 0; h < HR; ++h) acc[q][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[h], acc[q][h], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      bc[q] = bn[q];
      bn[q] = bnn[q];
    }
  }
#pragma unroll
  for (int q = 0; q < QM; ++q)
    if (q < nq) epi(wave + W * q, acc[q]);
}

template <int NL, bool GRAD, int W, int RT>
__global__ void __launch_bounds__(W * kWave) k_chain(ChainLaunch cl) {
  constexpr int R = kChainRows * RT;   // rows of this workgroup
  constexpr int HR = 2 * RT;
  const float inv_alpha = 1.f / cl.alpha, k_exp = 1.4426950408889634f * inv_alpha;
  extern __shared__ uint4 chain_lds[];
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
  const int l16 = lane & 15, kq = lane >> 4;
  // member-major logical order in chunks of row tiles per XCD: an XCD works
  // through a run of row tiles of one (member, species) network at a time,
  // whose weights then stay in its L2
  const int lb = xcd_chunked(blockIdx.x, cl.xcd_chunk);
  if (lb >= cl.n_blocks) return;
  const int n_rt = cl.n_blocks / cl.n_members;
  const int mb = lb / n_rt;
  const int r0 = (lb % n_rt) * R;
  int s = -1;
  for (int q = 0; q < cl.n_groups; ++q)
    if (r0 >= cl.bucket_off[q] && r0 < cl.bucket_off[q + 1]) s = q;
  if (s < 0) return;
  const ChainNet &net = cl.nets[mb * cl.n_groups + s];
  uint16_t *act[NL + 1];
#pragma unroll
  for (int l = 0; l <= NL; ++l) act[l] = (uint16_t *)((char *)chain_lds + (size_t)cl.lds_off[l] * RT);

  // h_0 tile (this member's slice of the first layer's output) into LDS
  {
    const int w0 = net.width[0], cpr = w0 / 8;
    const uint16_t *src = cl.H0 + (size_t)r0 * cl.ldh + (size_t)mb * cl.h_member_stride;
    for (int idx = tid; idx < R * cpr; idx += blockDim.x) {
      const int row = idx / cpr, ch = idx % cpr;
      *(uint4 *)(act[0] + row * cl.lds_ld[0] + ch * 8) = *(const uint4 *)(src + (size_t)row * cl.ldh + ch * 8);
    }
  }
  __syncthreads();

#pragma unroll
  for (int l = 1; l <= NL; ++l) {
    const int K = net.width[l - 1], N = net.width[l];
    const float *bias = net.b[l - 1];
    uint16_t *out = act[l];
    const int ldo = cl.lds_ld[l];
    if (l < NL) {
      chain_gemm<W, RT>(act[l - 1], cl.lds_ld[l - 1], K, net.W[l - 1], K, N, wave, lane,
                 [&](int cb, const floatx4_t *acc) {
                   const int col = cb * 16 + 4 * kq;
                   const float4 bc = *(const float4 *)(bias + col);
#pragma unroll
                   for (int h = 0; h < HR; ++h)
                     *(uint2 *)(out + (16 * h + l16) * ldo + col) =
                         pack4_bf16(celu_f(acc[h][0] + bc.x, cl.alpha, k_exp), celu_f(acc[h][1] + bc.y, cl.alpha, k_exp),
                                    celu_f(acc[h][2] + bc.z, cl.alpha, k_exp), celu_f(acc[h][3] + bc.w, cl.alpha, k_exp));
                 });
    } else {
      // last hidden layer: h_last (bfloat16) into its tile
      chain_gemm<W, RT>(act[l - 1], cl.lds_ld[l - 1], K, net.W[l - 1], K, N, wave, lane,
                 [&](int cb, const floatx4_t *acc) {
                   const int col = cb * 16 + 4 * kq;
                   const float4 bc = *(const float4 *)(bias + col);
#pragma unroll
                   for (int h = 0; h < HR; ++h)
                     *(uint2 *)(out + (16 * h + l16) * ldo + col) =
                         pack4_bf16(celu_f(acc[h][0] + bc.x, cl.alpha, k_exp), celu_f(acc[h][1] + bc.y, cl.alpha, k_exp),
                                    celu_f(acc[h][2] + bc.z, cl.alpha, k_exp), celu_f(acc[h][3] + bc.w, cl.alpha, k_exp));
                 });
    }
    __syncthreads();
  }

  // the member's energy of each row, E = h_last . w_out + b_out, and (for
  // forces) d_last = w_out CELU'(h_last) / M in place of h_last.  Eight
  // threads per row, each over the 8-column chunks seg, seg + 8, ..., then
  // summed over the eight: a fixed order, whatever the workgroup's shape.
  {
    const int N = net.width[NL], nch = N / 8, ldo = cl.lds_ld[NL];
    uint16_t *hl = act[NL];
    // R * 8 is a multiple of the workgroup size: every group of eight lanes
    // takes the loop's iterations together
    for (int t8 = tid; t8 < R * 8; t8 += W * kWave) {
      const int row = t8 >> 3, seg = t8 & 7;
      float e = 0.f;
      for (int ch = seg; ch < nch; ch += 8) {
        uint4 u = *(const uint4 *)(hl + row * ldo + ch * 8);
        const float4 w0 = *(const float4 *)(net.w_out + ch * 8);
        const float4 w1 = *(const float4 *)(net.w_out + ch * 8 + 4);
        const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
        uint16_t hv[8];
        *(uint4 *)hv = u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float h = from_bf16(hv[k]);
          e += h * wv[k];
          hv[k] = to_bf16(wv[k] * dcelu_h(h, inv_alpha) * cl.inv_m);
        }
        if (GRAD) *(uint4 *)(hl + row * ldo + ch * 8) = *(const uint4 *)hv;
      }
      e = sum8_dpp(e);
      if (seg == 0) {
        if (cl.n_members == 1) {
          // a single network: the row's energy is the atomic energy
          const int atom = cl.perm[r0 + row];
          if (atom >= 0) cl.e_atom[atom] = e + net.b_out;
        } else {
          cl.e_mem[(size_t)(r0 + row) * cl.n_members + mb] = e + net.b_out;
        }
      }
    }
    __syncthreads();
  }
  if (!GRAD) return;

  // backward: d_{l-1} = (d_l W_l) * CELU'(h_{l-1}), in place over h_{l-1}
#pragma unroll
  for (int l = NL; l >= 1; --l) {
    const int K = net.width[l], N = net.width[l - 1];
    uint16_t *hd = act[l - 1];
    const int ldo = cl.lds_ld[l - 1];
    chain_gemm<W, RT>(act[l], cl.lds_ld[l], K, net.Wt[l - 1], K, N, wave, lane,
               [&](int cb, const floatx4_t *acc) {
                 const int col = cb * 16 + 4 * kq;
#pragma unroll
                 for (int h = 0; h < HR; ++h) {
                   uint2 *p = (uint2 *)(hd + (16 * h + l16) * ldo + col);
                   const uint2 hv = *p;
                   *p = pack4_bf16(acc[h][0] * dcelu_h(__uint_as_float(hv.x << 16), inv_alpha),
                                   acc[h][1] * dcelu_h(__uint_as_float(hv.x & 0xffff0000u), inv_alpha),
                                   acc[h][2] * dcelu_h(__uint_as_float(hv.y << 16), inv_alpha),
                                   acc[h][3] * dcelu_h(__uint_as_float(hv.y & 0xffff0000u), inv_alpha));
                 }
               });
    __syncthreads();
  }

  // d_0 tile to global (16-byte stores)
  {
    const int w0 = net.width[0], cpr = w0 / 8;
    uint16_t *dst = cl.D0 + (size_t)r0 * cl.ldd + (size_t)mb * cl.d_member_stride;
    for (int idx = tid; idx < R * cpr; idx += blockDim.x) {
      const int row = idx / cpr, ch = idx % cpr;
      *(uint4 *)(dst + (size_t)row * cl.ldd + ch * 8) = *(const uint4 *)(act[0] + row * cl.lds_ld[0] + ch * 8);
    }
  }
}

// Atomic energies: mean over the members' energies of each row.  Rows past
// the last species bucket carry no atom (and no permutation entry).
__global__ void k_chain_mean(const float *__restrict__ e_mem, int M, const int *__restrict__ perm,
                             const int *__restrict__ bucket_off, int n_groups, int rows, float inv_m,
                             float *__restrict__ e_atom) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows || row >= bucket_off[n_groups]) return;
  const int atom = perm[row];
  if (atom < 0) return;
  float e = 0.f;
  for (int m = 0; m < M; ++m) e += e_mem[(size_t)row * M + m];
  e_atom[atom] = e * inv_m;
}

template <int W, int RT>
static void chain_t(const ChainLaunch &cl, int n_hidden, bool grad, unsigned blocks, size_t lds_bytes,
                    hipStream_t st) {
  blocks = xcd_grid(blocks, cl.xcd_chunk);
  if (n_hidden == 1) {
    if (grad) k_chain<1, true, W, RT><<<blocks, W * kWave, lds_bytes, st>>>(cl);
    else k_chain<1, false, W, RT><<<blocks, W * kWave, lds_bytes, st>>>(cl);
  } else if (n_hidden == 2) {
    if (grad) k_chain<2, true, W, RT><<<blocks, W * kWave, lds_bytes, st>>>(cl);
    else k_chain<2, false, W, RT><<<blocks, W * kWave, lds_bytes, st>>>(cl);
  } else {
    if (grad) k_chain<3, true, W, RT><<<blocks, W * kWave, lds_bytes, st>>>(cl);
    else k_chain<3, false, W, RT><<<blocks, W * kWave, lds_bytes, st>>>(cl);
  }
}

// lds_bytes: the activation tiles of 32 rows; rt = 2 takes 64 rows per
// workgroup (twice the LDS), rt = 1 32.  rows is a multiple of 128.
void launch_chain(ChainLaunch cl, int n_hidden, bool grad, int rows, size_t lds_bytes, int waves, int rt,
                  hipStream_t st) {
  const int R = kChainRows * (rt == 2 ? 2 : 1);
  const unsigned blocks = (unsigned)(rows / R * cl.n_members);
  if (blocks == 0) return;
  cl.n_blocks = (int)blocks;
  cl.xcd_chunk = 512 / R;   // 512 rows of one network per chunk
  if (rt == 2) {
    if (waves == 4) chain_t<4, 2>(cl, n_hidden, grad, blocks, 2 * lds_bytes, st);
    else chain_t<8, 2>(cl, n_hidden, grad, blocks, 2 * lds_bytes, st);
  } else {
    if (waves == 4) chain_t<4, 1>(cl, n_hidden, grad, blocks, lds_bytes, st);
    else chain_t<8, 1>(cl, n_hidden, grad, blocks, lds_bytes, st);
  }
  if (cl.n_members > 1)
    k_chain_mean<<<(rows + 255) / 256, 256, 0, st>>>(cl.e_mem, cl.n_members, cl.perm, cl.bucket_off, cl.n_groups,
                                                      rows, cl.inv_m, cl.e_atom);
}

}  // namespace nnp
