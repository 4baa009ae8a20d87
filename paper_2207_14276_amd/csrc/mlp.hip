// Element networks (section "Neural Network Potentials": one feed-forward
// network per element; the total energy is the sum of atomic energies,
// energy-decomposition equation) and the float64 per-system reductions.
//
// Dense layers are grouped GEMMs over species buckets: rows of one species
// are contiguous and padded to 128, so a 128-row tile always belongs to one
// network, and one launch covers all species and all ensemble members of one
// layer index (members side by side in the activation buffers).
//   C[rows, n_out] = sum over K segments of A[rows, seg] . B[n_out, seg]^T
// with a fused epilogue:
//     forward:  CELU(acc + bias)              -> hidden activations
//     backward: acc * CELU'(layer input)      -> input gradient
//     output:   acc * scale (float32)         -> dE/dG, ensemble summed along K
// Activations are stored in the operand type: float32 for the float32 model
// (v_mfma_f32_32x32x2_f32), bfloat16 for the bfloat16 model
// (v_mfma_f32_32x32x16_bf16, float32 accumulate).
// A workgroup of 4 waves computes a 128 x TN tile (TN = 128: 2 x 2 waves of
// 64 x 64, TN = 64: 4 x 1 waves of 32 x 64), K staged through double-buffered
// LDS.  Blocks are renumbered so that consecutive logical blocks (which share
// an A row tile) run on the same XCD and hit the same L2.
#include "internal.h"
#include "fixed.h"
#include "wave.h"

#include <algorithm>

namespace nnp {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float -> bfloat16, round to nearest even (one hardware conversion; two
// values per instruction when packed)
typedef __bf16 bf16x2_hw __attribute__((ext_vector_type(2)));
typedef float floatx2_hw __attribute__((ext_vector_type(2)));
__device__ inline uint32_t bf16_bits_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline uint32_t bf16x2_bits_rne(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2_hw){lo, hi}, bf16x2_hw));
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <bool BF16> struct Op;
template <> struct Op<false> {
  typedef float T;
  static __device__ inline float load(const float *p) { return *p; }
  static __device__ inline void store(float *p, float v) { *p = v; }
};
template <> struct Op<true> {
  typedef uint16_t T;
  static __device__ inline float load(const uint16_t *p) { return bf16_to_f(*p); }
  static __device__ inline void store(uint16_t *p, float v) { *p = (uint16_t)bf16_bits_rne(v); }
};

// CELU(z) = z for z > 0, else alpha (exp(z / alpha) - 1); inv_alpha = 1 / alpha.
__device__ inline float celu(float z, float alpha, float inv_alpha) {
  return z > 0.f ? z : alpha * expm1f(z * inv_alpha);
}
// The same with the hardware exp2 (about 1 ulp; the absolute error near
// z = 0 stays ~1e-7 alpha) for outputs rounded to bfloat16 next; k_exp =
// log2(e) / alpha.
__device__ inline float celu_bf16(float z, float alpha, float k_exp) {
  return z > 0.f ? z : alpha * (__builtin_amdgcn_exp2f(z * k_exp) - 1.f);
}

// CELU'(z) from h = CELU(z): 1 for h > 0, else exp(z / alpha) = 1 + h / alpha.
__device__ inline float dcelu_from_h(float h, float inv_alpha) { return h > 0.f ? 1.f : 1.f + h * inv_alpha; }


template <int EPI, bool BF16, int TN>
__global__ void __launch_bounds__(256) k_gemm(GemmLaunch gl) {
  const float inv_alpha = 1.f / gl.alpha, k_exp = 1.4426950408889634f * inv_alpha;
  typedef typename Op<BF16>::T T;
  constexpr int TM = kTileM;
  constexpr int TK = BF16 ? 32 : 16;
  constexpr int PAD = BF16 ? 8 : 1;          // row padding in elements
  constexpr int LD = TK + PAD;
  constexpr int WM = TN == 128 ? 64 : 32;    // wave tile rows
  constexpr int WN = 64;                     // wave tile cols
  constexpr int WAVES_N = TN / WN;
  constexpr int BM = WM / 32, BN = WN / 32;  // 32x32 MFMA blocks per wave
  constexpr int EPV = 16 / sizeof(T);        // elements per 16-byte vector
  constexpr int A_VEC = TM * TK / EPV / 256; // 16-byte loads per thread
  constexpr int B_VEC = TN * TK / EPV / 256;
  static_assert(A_VEC >= 1 && B_VEC >= 1, "tile too small");
  __shared__ __attribute__((aligned(16))) T smem[2][(TM + TN) * LD];

  // logical block -> (row tile, member, col tile); columns fastest
  const int lb = xcd_chunked(blockIdx.x, gl.xcd_chunk);
  if (lb >= gl.n_blocks) return;
  const int n_ct = gl.col_tiles;
  const int ct = lb % n_ct;
  const int mb = (lb / n_ct) % gl.n_members;
  const int rt = lb / (n_ct * gl.n_members);
  const int r0 = rt * TM;
  int s = -1;
  for (int q = 0; q < gl.n_groups; ++q)
    if (r0 >= gl.bucket_off[q] && r0 < gl.bucket_off[q + 1]) s = q;
  if (s < 0) return;
  const GemmGroup grp = gl.g[mb * gl.n_groups + s];
  const int c0 = ct * TN;
  if (c0 >= grp.n_out) return;
  const int K = grp.K;                 // per segment
  const int nseg = gl.n_seg;
  const int nk = (K + TK - 1) / TK;    // chunks per segment
  const int total = nk * nseg;

  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
  const int l32 = lane & 31, hi = lane >> 5;
  const int wr = wave / WAVES_N, wc = wave % WAVES_N;

  const T *A = (const T *)gl.A + (size_t)r0 * gl.lda + (size_t)mb * gl.a_member_stride;
  const T *B = (const T *)grp.B;
  const size_t ldb = grp.ldb ? (size_t)grp.ldb : (size_t)K * nseg;

  uint4 ra[A_VEC], rb[B_VEC];
  auto load_chunk = [&](int c) {
    const int seg = c / nk, k0 = (c % nk) * TK;
#pragma unroll
    for (int q = 0; q < A_VEC; ++q) {
      const int idx = q * 256 + tid;
      const int row = idx / (TK / EPV), cv = idx % (TK / EPV);
      const int k = k0 + cv * EPV;
      ra[q] = k < K ? *(const uint4 *)(A + (size_t)row * gl.lda + (size_t)seg * gl.a_seg_stride + k)
                    : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int q = 0; q < B_VEC; ++q) {
      const int idx = q * 256 + tid;
      const int row = idx / (TK / EPV), cv = idx % (TK / EPV);
      const int k = k0 + cv * EPV, col = c0 + row;
      rb[q] = (k < K && col < grp.n_out) ? *(const uint4 *)(B + (size_t)col * ldb + (size_t)seg * K + k)
                                         : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_chunk = [&](int buf) {
    T *As = smem[buf];
    T *Bs = As + TM * LD;
#pragma unroll
    for (int q = 0; q < A_VEC; ++q) {
      const int idx = q * 256 + tid;
      const int row = idx / (TK / EPV), cv = idx % (TK / EPV);
      if (BF16) {
        *(uint4 *)(As + row * LD + cv * EPV) = ra[q];
      } else {
        float *d = (float *)(As + row * LD + cv * EPV);
        d[0] = __uint_as_float(ra[q].x); d[1] = __uint_as_float(ra[q].y);
        d[2] = __uint_as_float(ra[q].z); d[3] = __uint_as_float(ra[q].w);
      }
    }
#pragma unroll
    for (int q = 0; q < B_VEC; ++q) {
      const int idx = q * 256 + tid;
      const int row = idx / (TK / EPV), cv = idx % (TK / EPV);
      if (BF16) {
        *(uint4 *)(Bs + row * LD + cv * EPV) = rb[q];
      } else {
        float *d = (float *)(Bs + row * LD + cv * EPV);
        d[0] = __uint_as_float(rb[q].x); d[1] = __uint_as_float(rb[q].y);
        d[2] = __uint_as_float(rb[q].z); d[3] = __uint_as_float(rb[q].w);
      }
    }
  };

  floatx16 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = floatx16{};

  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  for (int c = 0; c < total; ++c) {
    const int cur = c & 1;
    if (c + 1 < total) load_chunk(c + 1);
    const T *As = smem[cur];
    const T *Bs = As + TM * LD;
    if (BF16) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 16) {
        bf16x8 a[BM], b[BN];
#pragma unroll
        for (int i = 0; i < BM; ++i)
          a[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)(As + (wr * WM + i * 32 + l32) * LD + kk + 8 * hi));
#pragma unroll
        for (int j = 0; j < BN; ++j)
          b[j] = __builtin_bit_cast(bf16x8, *(const uint4 *)(Bs + (wc * WN + j * 32 + l32) * LD + kk + 8 * hi));
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 2) {
        float a[BM], b[BN];
#pragma unroll
        for (int i = 0; i < BM; ++i) a[i] = ((const float *)As)[(wr * WM + i * 32 + l32) * LD + kk + hi];
#pragma unroll
        for (int j = 0; j < BN; ++j) b[j] = ((const float *)Bs)[(wc * WN + j * 32 + l32) * LD + kk + hi];
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    if (c + 1 < total) store_chunk(cur ^ 1);
    __syncthreads();
  }

  // D[row][col]: col = lane % 32, row = 8 (i / 4) + 4 (lane / 32) + i % 4
#pragma unroll
  for (int bj = 0; bj < BN; ++bj) {
    const int col = c0 + wc * WN + bj * 32 + l32;
    if (col >= grp.n_out) continue;
    const float bias = EPI == kEpiFwd ? grp.bias[col] : 0.f;
#pragma unroll
    for (int bi = 0; bi < BM; ++bi) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int row = r0 + wr * WM + bi * 32 + 8 * (i / 4) + 4 * hi + (i % 4);
        const float v = acc[bi][bj][i];
        if (EPI == kEpiFwd) {
          T *out = (T *)gl.C + (size_t)row * gl.ldc + (size_t)mb * gl.c_member_stride + col;
          Op<BF16>::store(out, BF16 ? celu_bf16(v + bias, gl.alpha, k_exp) : celu(v + bias, gl.alpha, inv_alpha));
        } else if (EPI == kEpiBwd) {
          T *out = (T *)gl.C + (size_t)row * gl.ldc + (size_t)mb * gl.c_member_stride + col;
          const float h = Op<BF16>::load((const T *)gl.H + (size_t)row * gl.ldh +
                                         (size_t)mb * gl.h_member_stride + col);
          Op<BF16>::store(out, v * dcelu_from_h(h, inv_alpha) * gl.scale);
        } else {
          float *out = (float *)gl.C + (size_t)row * gl.ldc + col;
          *out = v * gl.scale;
        }
      }
    }
  }
}

// Eight consecutive elements in one 16-byte (bfloat16) or two 16-byte
// (float32) accesses; p is 16-byte aligned.
template <bool BF16> struct Vec8;
template <> struct Vec8<true> {
  static __device__ inline void load(const uint16_t *p, float v[8]) {
    const uint4 u = *(const uint4 *)p;
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = __uint_as_float(w[q] << 16);
      v[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
    }
  }
  static __device__ inline void store(uint16_t *p, const float v[8]) {
    uint4 u;
    u.x = bf16x2_bits_rne(v[0], v[1]);
    u.y = bf16x2_bits_rne(v[2], v[3]);
    u.z = bf16x2_bits_rne(v[4], v[5]);
    u.w = bf16x2_bits_rne(v[6], v[7]);
    *(uint4 *)p = u;
  }
};
template <> struct Vec8<false> {
  static __device__ inline void load(const float *p, float v[8]) {
    const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
  static __device__ inline void store(float *p, const float v[8]) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
    *(float4 *)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  }
};

// bfloat16 GEMM fed by direct global -> LDS loads (global_load_lds_dwordx4):
// no staging registers and no LDS store instructions, so a three-stage ring
// fits in the register budget of the two-stage kernel above.  Each 128 x 32
// (or TN x 32) operand tile is 16-byte slots, row r's 4 K-chunks at slots
// 4 r + (chunk ^ swz(r)); a wave's load instruction fills 64 consecutive
// slots, and the XOR swizzle keeps the MFMA operand reads free of bank
// conflicts for both 8- and 16-lane LDS phases.  Requires every K (per
// segment), lda, ldb and the segment and member offsets to be multiples of
// 32 elements (gl.k32); column tiles past n_out read a clamped, valid row and
// their results are discarded.
__device__ inline int lds_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

// s_waitcnt immediate: vmcnt = n (bits 3:0 and 15:14), expcnt and lgkmcnt
// left at their maxima.
constexpr int vm_imm(int n) { return 0xF70 | (n & 15) | ((n >> 4) << 14); }

// Waits until at most `ahead` chunks' worth of this wave's loads (LOADS
// instructions per chunk) are outstanding; ahead is wave-uniform.
template <int LOADS, int MAXA>
__device__ inline void wait_chunks(int ahead) {
  if (MAXA >= 3 && ahead >= 3) __builtin_amdgcn_s_waitcnt(vm_imm(3 * LOADS));
  else if (MAXA >= 2 && ahead >= 2) __builtin_amdgcn_s_waitcnt(vm_imm(2 * LOADS));
  else if (MAXA >= 1 && ahead >= 1) __builtin_amdgcn_s_waitcnt(vm_imm(LOADS));
  else __builtin_amdgcn_s_waitcnt(vm_imm(0));
}

// Bits 0, 2, 4, ... of x gathered into bits 0, 1, 2, ...
__device__ inline unsigned long long even_bits(unsigned long long x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0f0f0f0f0f0f0f0full;
  x = (x | (x >> 4)) & 0x00ff00ff00ff00ffull;
  x = (x | (x >> 8)) & 0x0000ffff0000ffffull;
  return (x | (x >> 16)) & 0x00000000ffffffffull;
}

// 256-wide tiles hold 128 accumulator registers per lane; the kernel is
// held to 256 registers in all so that two workgroups share a compute unit.
// STAGES: depth of the operand ring; loads run STAGES - 1 chunks ahead.
template <int EPI, int TN, bool SPAN, int STAGES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TN == 256 ? 2 : 1)))
k_gemm_dl(GemmLaunch gl) {
  const float inv_alpha = 1.f / gl.alpha, k_exp = 1.4426950408889634f * inv_alpha;
  typedef uint16_t T;
  constexpr int TM = kTileM;
  constexpr int TK = 32;
  static_assert(STAGES == 3, "ring depth: the first two chunks are issued unconditionally");
  constexpr int WM = TN == 64 ? 32 : 64;
  constexpr int WN = TN == 256 ? 128 : 64;
  constexpr int WAVES_N = TN / WN;
  constexpr int BM = WM / 32, BN = WN / 32;
  constexpr int A_SLOTS = TM * 4, B_SLOTS = TN * 4;  // 16-byte slots per stage
  constexpr int A_LD = A_SLOTS / 256, B_LD = B_SLOTS / 256;
  constexpr int LOADS = A_LD + B_LD;                  // load instructions per chunk and thread
  static_assert(A_LD >= 1 && B_LD >= 1, "tile too small");
  __shared__ __attribute__((aligned(16))) uint4 smem[STAGES][A_SLOTS + B_SLOTS];

  const int lb = xcd_chunked(blockIdx.x, gl.xcd_chunk);
  if (lb >= gl.n_blocks) return;
  const int n_ct = gl.col_tiles;
  const int ct = lb % n_ct;
  // SPAN: the output columns of all members side by side (member-major), one
  // column space of n_members * n_out; every member reads the same A
  const int mb = SPAN ? 0 : (lb / n_ct) % gl.n_members;
  const int rt = SPAN ? lb / n_ct : lb / (n_ct * gl.n_members);
  const int r0 = rt * TM;
  // the row tile's species bucket, and (with row records) where its real
  // rows end
  int s = -1, real_end = 0;
  for (int q = 0; q < gl.n_groups; ++q)
    if (r0 >= gl.bucket_off[q] && r0 < gl.bucket_off[q + 1]) {
      s = q;
      if (gl.row_mask) real_end = gl.bucket_off[q] + gl.bucket_cnt[q];
    }
  if (s < 0) return;
  const GemmGroup grp = gl.g[mb * gl.n_groups + s];
  const int n_cols = SPAN ? grp.n_out * gl.n_members : grp.n_out;
  const int c0 = ct * TN;
  if (c0 >= n_cols) return;
  const int K = grp.K;
  const int nseg = gl.n_seg;
  const int nk = K / TK;

  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
  const int l32 = lane & 31, hi = lane >> 5;
  const int wr = wave / WAVES_N, wc = wave % WAVES_N;

  const T *A = (const T *)gl.A + (size_t)r0 * gl.lda + (size_t)mb * gl.a_member_stride;
  const T *B = (const T *)grp.B;
  const size_t ldb = grp.ldb ? (size_t)grp.ldb : (size_t)K * nseg;

  // this thread's source rows and chunks (fixed over the K loop)
  const T *asrc[A_LD];
  const T *bsrc[B_LD];
#pragma unroll
  for (int q = 0; q < A_LD; ++q) {
    const int sl = q * 256 + tid, row = sl >> 2, kc = (sl & 3) ^ lds_swz(row);
    asrc[q] = A + (size_t)row * gl.lda + kc * 8;
  }
#pragma unroll
  for (int q = 0; q < B_LD; ++q) {
    const int sl = q * 256 + tid, row = sl >> 2, kc = (sl & 3) ^ lds_swz(row);
    const int col = min(c0 + row, n_cols - 1);
    if (SPAN) {
      const int m = col / grp.n_out;
      bsrc[q] = (const T *)gl.g[m * gl.n_groups + s].B + (size_t)(col - m * grp.n_out) * ldb + kc * 8;
    } else {
      bsrc[q] = B + (size_t)col * ldb + kc * 8;
    }
  }
  auto issue = [&](int c, int stage) {
    const int seg = c / nk, k0 = (c % nk) * TK;
    const size_t ao = (size_t)seg * gl.a_seg_stride + k0, bo = (size_t)seg * K + k0;
#pragma unroll
    for (int q = 0; q < A_LD; ++q)
      __builtin_amdgcn_global_load_lds((const void *)(asrc[q] + ao),
                                       (__attribute__((address_space(3))) void *)&smem[stage][q * 256 + wave * kWave],
                                       16, 0, 0);
#pragma unroll
    for (int q = 0; q < B_LD; ++q)
      __builtin_amdgcn_global_load_lds((const void *)(bsrc[q] + bo),
                                       (__attribute__((address_space(3))) void *)&smem[stage][A_SLOTS + q * 256 + wave * kWave],
                                       16, 0, 0);
  };

  floatx16 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = floatx16{};

  // The AEV halves (16 columns) that some row of the tile may have
  // non-zero (wave-uniform; all without the record).  First layer: after
  // the first chunks, a K chunk (halves 2c, 2c + 1) is loaded only if one
  // of its halves is live, and a half's MFMAs run only if it is; the
  // skipped products are zero for every row.  dE/dG: a column half no row
  // has is read by no one and is not stored; a wave whose columns are all
  // such runs no MFMAs.  Each wave loads the tile's row records (1 KB, two
  // per lane) like the operands, ahead of chunk 0, into its own slots of the
  // ring's last stage, which chunk 2 fills only after the records are read.
  constexpr bool kMaskK = EPI == kEpiFwd, kMaskN = EPI == kEpiOut;
  const bool masked = gl.row_mask != nullptr && (kMaskN || (kMaskK && nseg == 1 && nk <= 32));
  static_assert(TM == 2 * kWave && A_SLOTS >= 256, "two row records per lane, in the wave's A slots");
  if (masked)
    __builtin_amdgcn_global_load_lds((const void *)(gl.row_mask + r0 + 2 * lane),
                                     (__attribute__((address_space(3))) void *)&smem[STAGES - 1][wave * kWave],
                                     16, 0, 0);
  // the first chunks go out in order (every call has at least STAGES - 1)
  const int n_pro = STAGES - 1;
#pragma unroll
  for (int q = 0; q < STAGES - 1; ++q) issue(q, q);
  unsigned long long live_h = ~0ull;
  // live K chunks after the first ones, in order (first layer, masked: one
  // segment of at most 32 chunks), set with live_h
  unsigned long long kc_issue = 0, kc_comp = 0;
  int total = kMaskK && masked ? n_pro : nk * nseg;  // masked first layer: until live_h is known
  // chunk of the k-th issue (called for k = 0, 1, 2, ... in turn)
  auto chunk_at = [&](int k) {
    if (!(kMaskK && masked) || k < n_pro) return k;
    const int cc = __builtin_ctzll(kc_issue);
    kc_issue &= kc_issue - 1;
    return cc;
  };
  bool wave_live = true;  // whether any column half of this wave is live (dE/dG)
  bool some_dead = false;  // whether a column half of the tile is not (dE/dG)

  for (int c = 0; c < total; ++c) {
    // this wave's loads of chunk c are done once at most those of the
    // chunks issued after it remain
    wait_chunks<LOADS, STAGES - 2>(min(total - 1 - c, STAGES - 2));
    if (masked && c == 0) {
      // this wave's own record load preceded its chunk 0 loads, waited for
      // above (no barrier needed); the read waits for itself (a plain LDS
      // read here would make the compiler wait for every load in flight)
      uint4 r;
      const unsigned ra =
          (unsigned)(uintptr_t)(__attribute__((address_space(3))) uint4 *)&smem[STAGES - 1][wave * kWave + lane];
      asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(r) : "v"(ra) : "memory");
      // records past the bucket's real rows are not the forward's
      const int real = real_end - r0 - 2 * lane;
      const unsigned h_lo = (real > 0 ? r.x : 0u) | (real > 1 ? r.z : 0u);
      const unsigned h_hi = (real > 0 ? r.y : 0u) | (real > 1 ? r.w : 0u);
      live_h = ((unsigned long long)wave_or(h_hi) << 32) | wave_or(h_lo);
      if (kMaskN) {
        // a column tile without a live half: nothing to compute or store
        // (every wave leaves here; the operand loads in flight land in this
        // workgroup's LDS first)
        const unsigned long long tile_h = (live_h >> (c0 / 16)) & ((1ull << (TN / 16 - 1) << 1) - 1);
        if (tile_h == 0) {
          __builtin_amdgcn_s_waitcnt(vm_imm(0));
          return;
        }
        // every half of the column tile live: stores without the check
        some_dead = tile_h != ((1ull << (TN / 16 - 1) << 1) - 1);
        wave_live = ((live_h >> ((c0 + wc * WN) / 16)) & ((1ull << (WN / 16 - 1) << 1) - 1)) != 0;
      } else {
        kc_issue = even_bits(live_h | (live_h >> 1)) & (nk >= 64 ? ~0ull : (1ull << nk) - 1) &
                   ~((1ull << n_pro) - 1);
        kc_comp = kc_issue;
        total = n_pro + __builtin_popcountll(kc_issue);
      }
    }
    // a plain barrier: LDS is coherent within the workgroup, every wave has
    // waited for its own part of chunk c above, and its reads of the stage
    // overwritten next were consumed (by MFMAs) before it got here; a full
    // __syncthreads() would also wait for the loads of later chunks
    __builtin_amdgcn_s_barrier();
    // stage (c + STAGES - 1) % STAGES was last read for chunk c - 1, which
    // every wave has finished (barrier above)
    if (c + STAGES - 1 < total) issue(chunk_at(c + STAGES - 1), (c + STAGES - 1) % STAGES);
    const uint4 *As = smem[c % STAGES];
    const uint4 *Bs = As + A_SLOTS;
    // live halves of this chunk (first layer, masked)
    unsigned halves = 3u;
    if (kMaskK && masked) {
      int cc = c;
      if (c >= n_pro) {
        cc = __builtin_ctzll(kc_comp);
        kc_comp &= kc_comp - 1;
      }
      halves = (unsigned)(live_h >> (2 * cc)) & 3u;
    }
    if (!wave_live) continue;
#pragma unroll
    for (int kk = 0; kk < TK; kk += 16) {
      if (!((halves >> (kk / 16)) & 1u)) continue;
      const int ch = kk / 8 + hi;
      bf16x8 a[BM], b[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        const int r = wr * WM + i * 32 + l32;
        a[i] = __builtin_bit_cast(bf16x8, As[4 * r + (ch ^ lds_swz(r))]);
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int r = wc * WN + j * 32 + l32;
        b[j] = __builtin_bit_cast(bf16x8, Bs[4 * r + (ch ^ lds_swz(r))]);
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }

  // Epilogue through LDS: each 32 x 32 accumulator block is written to a
  // per-wave LDS tile in the MFMA layout (col = lane % 32, row = 8 (i / 4) +
  // 4 (lane / 32) + i % 4) and read back by rows, so that every global access
  // moves 8 consecutive elements (16-byte bfloat16 rows, 2 x 16-byte float32
  // rows).  Output widths are multiples of 8: an 8-column chunk is either
  // wholly inside n_out or wholly outside.
  if constexpr (EPI == kEpiOut) {
    // float32 output: straight from the accumulators, whose layout already
    // gives each half-wave 32 consecutive columns (128 bytes) of one row
#pragma unroll
    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
      for (int bj = 0; bj < BN; ++bj) {
        const int col = c0 + wc * WN + bj * 32 + l32;
        if (col >= n_cols || (some_dead && !((live_h >> (col / 16)) & 1ull))) continue;
        float *out = (float *)gl.C + (size_t)(r0 + wr * WM + bi * 32 + 4 * hi) * gl.ldc + col;
#pragma unroll
        for (int i = 0; i < 16; ++i) out[(size_t)(8 * (i / 4) + (i % 4)) * gl.ldc] = acc[bi][bj][i] * gl.scale;
      }
    return;
  }
  constexpr int EP_LD = 36;                     // floats per LDS row (16-byte aligned)
  __syncthreads();                              // every wave is done with the operand tiles
  float *ep = (float *)smem + wave * 32 * EP_LD;
#pragma unroll
  for (int bi = 0; bi < BM; ++bi) {
#pragma unroll
    for (int bj = 0; bj < BN; ++bj) {
#pragma unroll
      for (int i = 0; i < 16; ++i) ep[(8 * (i / 4) + 4 * hi + (i % 4)) * EP_LD + l32] = acc[bi][bj][i];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int chunk = q * kWave + lane;     // 128 chunks of 8: 32 rows x 4
        const int rr = chunk >> 2, cc = (chunk & 3) * 8;
        const int row = r0 + wr * WM + bi * 32 + rr;
        const int vcol = c0 + wc * WN + bj * 32 + cc;
        if (vcol >= n_cols) continue;
        // the member and its column (8-column chunks never straddle members:
        // output widths are multiples of 8)
        const int om = SPAN ? vcol / grp.n_out : mb;
        const int col = SPAN ? vcol - om * grp.n_out : vcol;
        float v[8];
        const float4 v0 = *(const float4 *)(ep + rr * EP_LD + cc);
        const float4 v1 = *(const float4 *)(ep + rr * EP_LD + cc + 4);
        v[0] = v0.x; v[1] = v0.y; v[2] = v0.z; v[3] = v0.w;
        v[4] = v1.x; v[5] = v1.y; v[6] = v1.z; v[7] = v1.w;
        if (EPI == kEpiFwd) {
          float b[8];
          Vec8<false>::load((SPAN ? gl.g[om * gl.n_groups + s].bias : grp.bias) + col, b);
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = celu_bf16(v[e] + b[e], gl.alpha, k_exp);
          Vec8<true>::store((T *)gl.C + (size_t)row * gl.ldc + (size_t)om * gl.c_member_stride + col, v);
        } else if (EPI == kEpiBwd) {
          float h[8];
          Vec8<true>::load((const T *)gl.H + (size_t)row * gl.ldh + (size_t)mb * gl.h_member_stride + col, h);
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = v[e] * dcelu_from_h(h[e], inv_alpha) * gl.scale;
          Vec8<true>::store((T *)gl.C + (size_t)row * gl.ldc + (size_t)mb * gl.c_member_stride + col, v);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] *= gl.scale;
          Vec8<false>::store((float *)gl.C + (size_t)row * gl.ldc + col, v);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// operand ring depth per tile width
constexpr int kStages128 = 3, kStages256 = 3;

template <int EPI, bool BF16>
static void launch_t(GemmLaunch gl, int row_tiles, int tn, hipStream_t st) {
  // the blocks of one row tile (every column tile and member) form a chunk
  gl.xcd_chunk = (gl.span ? 1 : gl.n_members) * gl.col_tiles;
  gl.n_blocks = row_tiles * gl.xcd_chunk;
  const unsigned blocks = xcd_grid((unsigned)gl.n_blocks, gl.xcd_chunk);
  if (BF16 && gl.k32) {
    if constexpr (EPI == kEpiFwd) {
      if (gl.span) {
        k_gemm_dl<EPI, 256, true, kStages256><<<blocks, 256, 0, st>>>(gl);
        return;
      }
    }
    if (tn == 256) k_gemm_dl<EPI, 256, false, kStages256><<<blocks, 256, 0, st>>>(gl);
    else if (tn == 128) k_gemm_dl<EPI, 128, false, kStages128><<<blocks, 256, 0, st>>>(gl);
    else k_gemm_dl<EPI, 64, false, 3><<<blocks, 256, 0, st>>>(gl);
    return;
  }
  if (tn == 256) tn = 128;
  if (tn == 128) k_gemm<EPI, BF16, 128><<<blocks, 256, 0, st>>>(gl);
  else k_gemm<EPI, BF16, 64><<<blocks, 256, 0, st>>>(gl);
}

// Whether every member of a species group has the same output width, K and
// B row stride (the members-side-by-side tiling needs it).
static bool gemm_span_uniform(const GemmLaunch &gl) {
  for (int s = 0; s < gl.n_groups; ++s) {
    const GemmGroup &g0 = gl.g[s];
    for (int m = 1; m < gl.n_members; ++m) {
      const GemmGroup &g = gl.g[m * gl.n_groups + s];
      if (g.n_out != g0.n_out || g.K != g0.K || g.ldb != g0.ldb || !g.B != !g0.B) return false;
    }
  }
  return true;
}

// Whether every K chunk of 32 elements and every operand row start is
// 16-byte aligned and inside its row, and every output sums at least two
// chunks (the first two are loaded unconditionally), as the direct-to-LDS
// kernel needs.
static bool gemm_k32(const GemmLaunch &gl) {
  auto m32 = [](long long v) { return v % 32 == 0; };
  if (!m32(gl.lda) || !m32(gl.a_member_stride) || !m32(gl.a_seg_stride)) return false;
  for (int q = 0; q < gl.n_members * gl.n_groups; ++q) {
    const GemmGroup &g = gl.g[q];
    if (!g.B) continue;
    const long long ldb = g.ldb ? g.ldb : (long long)g.K * gl.n_seg;
    if (!m32(g.K) || !m32(ldb) || g.K * gl.n_seg < 64) return false;
  }
  return true;
}

void launch_gemm(int epi, bool bf16, GemmLaunch gl, int row_tiles, int max_n_out, int tn_pref, hipStream_t st) {
  if (row_tiles <= 0) return;
  gl.k32 = bf16 && gemm_k32(gl) ? 1 : 0;
  // 256-wide tiles (direct-to-LDS kernel only); for a forward layer whose
  // members all read the same input, the members' columns side by side
  const bool wide_ok = gl.k32 && max_n_out >= 160;
  const bool span_ok = wide_ok && epi == kEpiFwd && gl.a_member_stride == 0 && gemm_span_uniform(gl);
  // the tuned width, else: 256 for the AEV-gradient GEMM when that still
  // gives several workgroups per compute unit; 128-wide column tiles when
  // they waste little; else 64
  const int t128 = (max_n_out + 127) / 128 * 128, t64 = (max_n_out + 63) / 64 * 64;
  int tn = tn_pref == 64 || tn_pref == 128 || tn_pref == 256 ? tn_pref
         : wide_ok && epi == kEpiOut && row_tiles * ((max_n_out + 255) / 256) >= 2048 ? 256
         : (t128 - max_n_out) * 4 <= max_n_out && t128 <= t64 + 32 ? 128 : 64;
  if (tn == 256 && !wide_ok) tn = 128;
  gl.span = tn == 256 && span_ok ? 1 : 0;
  int cols = max_n_out;
  if (gl.span) {
    cols = 0;
    for (int s = 0; s < gl.n_groups; ++s)
      if (gl.g[s].B) cols = std::max(cols, gl.g[s].n_out * gl.n_members);
  }
  gl.col_tiles = (cols + tn - 1) / tn;
  if (bf16) {
    if (epi == kEpiFwd) launch_t<kEpiFwd, true>(gl, row_tiles, tn, st);
    else if (epi == kEpiBwd) launch_t<kEpiBwd, true>(gl, row_tiles, tn, st);
    else launch_t<kEpiOut, true>(gl, row_tiles, tn, st);
  } else {
    if (epi == kEpiFwd) launch_t<kEpiFwd, false>(gl, row_tiles, tn, st);
    else if (epi == kEpiBwd) launch_t<kEpiBwd, false>(gl, row_tiles, tn, st);
    else launch_t<kEpiOut, false>(gl, row_tiles, tn, st);
  }
}

// Output layer (one unit) of every ensemble member: E_row = mean over members
// of w . h + b, and dE/dh = w * CELU'(h) / M per member (or, for networks
// without hidden layers, dE/dG = mean of w).  One half-wave (32 lanes) per
// row; a lane takes 8 consecutive inputs at a time (one 16-byte bfloat16 or
// two 16-byte float32 accesses).  Hidden widths and the AEV length are
// multiples of 8, so a lane's 8 inputs never straddle a member's slice.
template <bool BF16>
__global__ void __launch_bounds__(256) k_energy(EnergyLaunch el, int rows) {
  const float inv_alpha = 1.f / el.alpha;
  typedef typename Op<BF16>::T T;
  const int half = threadIdx.x >> 5, l32 = threadIdx.x & 31;
  const int row = blockIdx.x * 8 + half;
  int s = -1;
  if (row < rows)
    for (int q = 0; q < el.n_groups; ++q)
      if (row >= el.bucket_off[q] && row < el.bucket_off[q + 1]) s = q;
  const int atom = s >= 0 ? el.perm[row] : -1;
  const bool active = atom >= 0;   // uniform over the half-wave
  float e = 0.f, bsum = 0.f;
  if (active) {
    const int K = el.K[s];
    for (int m = 0; m < el.n_members; ++m) {
      const float *w = el.w[m * el.n_groups + s];
      bsum += el.b[m * el.n_groups + s][0];
      const T *h = (const T *)el.Hin + (size_t)row * el.ldh + (size_t)m * el.h_member_stride;
      for (int k0 = 8 * l32; k0 < K; k0 += 256) {
        float hv[8], wv[8];
        Vec8<BF16>::load(h + k0, hv);
        Vec8<false>::load(w + k0, wv);
#pragma unroll
        for (int q = 0; q < 8; ++q) e += hv[q] * wv[q];
        if (el.want_grad) {
          if (el.hidden) {
            float gv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) gv[q] = wv[q] * dcelu_from_h(hv[q], inv_alpha) * el.inv_m;
            Vec8<BF16>::store((T *)el.Gout + (size_t)row * el.ldg + (size_t)m * el.g_member_stride + k0, gv);
          } else {
            // no hidden layer: dE/dG = mean of w, float32
            float *go = (float *)el.Gout + (size_t)row * el.ldg + k0;
            float gv[8];
            if (m > 0) Vec8<false>::load(go, gv);
#pragma unroll
            for (int q = 0; q < 8; ++q) gv[q] = (m == 0 ? 0.f : gv[q]) + wv[q] * el.inv_m;
            Vec8<false>::store(go, gv);
          }
        }
      }
    }
  }
  for (int off = 16; off >= 1; off >>= 1) e += __shfl_xor(e, off, 32);
  if (active && l32 == 0) el.e_atom[atom] = (e + bsum) * el.inv_m;
}

void launch_energy(const EnergyLaunch &el, bool bf16, int rows, hipStream_t st) {
  if (rows <= 0) return;
  if (bf16) k_energy<true><<<(rows + 7) / 8, 256, 0, st>>>(el, rows);
  else k_energy<false><<<(rows + 7) / 8, 256, 0, st>>>(el, rows);
}

// Per-system totals in float64: energies (sum of atomic energies) and the
// virial (sum of per-centre virials).  Deterministic two-level sum: fixed
// chunks of at most 4096 atoms, then the chunks of each system in order.
constexpr int kChunk = 4096;

__global__ void __launch_bounds__(256)
k_reduce_partial(const float *__restrict__ e_atom, const float *__restrict__ W_atom,
                 const SysDesc *__restrict__ sys, const int *__restrict__ chunk_sys,
                 const int *__restrict__ chunk_begin, double *__restrict__ partial,
                 double *__restrict__ energy, double *__restrict__ virial,
                 const unsigned long long *__restrict__ Ffix, float *__restrict__ F, Live n_chunks) {
  __shared__ double red[10][256 / kWave];
  const int ch = blockIdx.x;
  if (ch >= n_chunks.get()) return;  // the whole workgroup
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
  // fixed-point forces of the chunk's atoms (slots in launch order) to float32
  if (Ffix) {
    const int s3 = 3 * fix_shift(d);
    for (int t = 3 * b + threadIdx.x; t < 3 * e; t += blockDim.x) F[t] = from_fix((long long)Ffix[t + s3]);
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
    if (energy) {
      // one chunk per system (chunk ch is system ch): the sums are final
      if (threadIdx.x == 0) energy[ch] = v;
      else if (virial) virial[(size_t)9 * ch + threadIdx.x - 1] = v;
    } else {
      partial[(size_t)10 * ch + threadIdx.x] = v;
    }
  }
}

__global__ void k_reduce_final(const double *__restrict__ partial, const int *__restrict__ sys_chunk_off,
                               Live n_sys, double *__restrict__ energy, double *__restrict__ virial) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys.get()) return;
  double acc[10];
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int ch = sys_chunk_off[s]; ch < sys_chunk_off[s + 1]; ++ch)
    for (int q = 0; q < 10; ++q) acc[q] += partial[(size_t)10 * ch + q];
  energy[s] = acc[0];
  if (virial)
    for (int q = 0; q < 9; ++q) virial[(size_t)9 * s + q] = acc[1 + q];
}

void launch_reduce(const float *e_atom, const float *W_atom, const SysDesc *sys, Live n_sys,
                   const int *chunk_sys, const int *chunk_begin, Live n_chunks,
                   const int *sys_chunk_off, bool direct, double *partial, double *energy,
                   double *virial, const unsigned long long *Ffix, float *F, hipStream_t st) {
  // direct: every system exactly one chunk (chunk s is system s), the chunk
  // sums are the system sums, no second pass
  if (n_chunks.v > 0)
    k_reduce_partial<<<n_chunks.v, 256, 0, st>>>(e_atom, W_atom, sys, chunk_sys, chunk_begin, partial,
                                                 direct ? energy : nullptr, direct ? virial : nullptr, Ffix, F,
                                                 n_chunks);
  if (n_sys.v > 0 && !direct)
    k_reduce_final<<<(n_sys.v + 127) / 128, 128, 0, st>>>(partial, sys_chunk_off, n_sys, energy, virial);
}

}  // namespace nnp
