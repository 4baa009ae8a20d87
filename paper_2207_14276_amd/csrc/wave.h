// Wave-level helpers shared by the per-centre kernels (wave64).
#pragma once

#include "internal.h"
#include "fixed.h"

namespace nnp {

__device__ inline unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
}

// Hardware reciprocal and square root (about 1 ulp), in place of the
// correctly rounded division and square-root sequences.
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Neighbour vector d = r_j + image * L - r_i of entry e of centre i.
__device__ inline float4 entry_vec(const float4 &pi, const float4 &pj, int code, const float L[3]) {
  int ix, iy, iz;
  unpack_image(code, ix, iy, iz);
  float dx = (pj.x - pi.x) + (float)ix * L[0];
  float dy = (pj.y - pi.y) + (float)iy * L[1];
  float dz = (pj.z - pi.z) + (float)iz * L[2];
  return make_float4(dx, dy, dz, fast_sqrt(dx * dx + dy * dy + dz * dz));
}

// Lane reductions on the VALU (DPP) rather than through the LDS crossbar.
template <int CTRL, int ROWS = 0xF> __device__ inline float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
// sum over aligned groups of 4 / 8 / 16 lanes, result in every lane of the group
__device__ inline float sum4(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  return v;
}
__device__ inline float sum8(float v) {
  v = sum4(v);
  v += dpp<0x141>(v);  // row_half_mirror: quads 0 <-> 1 of each half-row
  return v;
}
__device__ inline float sum16(float v) {
  v = sum8(v);
  v += dpp<0x140>(v);  // row_mirror: halves 0 <-> 1 of each row
  return v;
}
// sum over the whole wave, returned in every lane
__device__ inline float wave_sum(float v) {
  v = sum16(v);
  v += dpp<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
  v += dpp<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// OR over the whole wave, returned in every lane (the steps of wave_sum)
template <int CTRL, int ROWS = 0xF> __device__ inline unsigned dpp_u(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
__device__ inline unsigned wave_or(unsigned v) {
  v |= dpp_u<0xB1>(v);
  v |= dpp_u<0x4E>(v);
  v |= dpp_u<0x141>(v);
  v |= dpp_u<0x140>(v);
  v |= dpp_u<0x142, 0xA>(v);
  v |= dpp_u<0x143, 0xC>(v);
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Orders this wave's LDS writes before its later LDS reads by other lanes
// (LDS requests of one wave are served in order; this only stops the
// compiler from moving accesses across it).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace nnp
