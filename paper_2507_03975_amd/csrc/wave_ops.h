// wave_ops.h -- small gfx950 building blocks shared by the wavefront kernels:
// a reciprocal refined to about one ulp, lane shifts across a 64-wide wave
// (DPP), and raw buffer resources whose out-of-range accesses are dropped.
#pragma once
#include <hip/hip_runtime.h>

namespace gsis {
namespace {

// 1/x: the hardware estimate refined by two Newton steps
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Lane shifts of a double across the wave: shr1 moves lane l's value to
// lane l + 1 (lane 0 keeps its own, or fill), shl1 to lane l - 1.
__device__ inline double shr1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double shl1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// shr1 with lane 0 taking fill (its own lane's fill) instead
__device__ inline double shr1_fill(double v, double fill) {
  int lo = __double2loint(fill), hi = __double2hiint(fill);
  lo = __builtin_amdgcn_update_dpp(lo, __double2loint(v), 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// lane l's value, l wave-uniform
__device__ inline double rdlane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
// shl1 with lane 63 taking fill instead
__device__ inline double shl1_fill(double v, double fill) {
  int lo = __double2loint(fill), hi = __double2hiint(fill);
  lo = __builtin_amdgcn_update_dpp(lo, __double2loint(v), 0x130, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(hi, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Raw buffer stores (gfx9 resource word 3 = 0x00020000): a store whose byte
// offset lies outside the resource's range is dropped by the hardware, so a
// lane with no cell issues the same instruction as the others and no branch
// splits a step (the load/store counters then stay exact for the waits).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kNoCell = 0x7ffffff0u;     // beyond every resource's range
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
__device__ inline void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
__device__ inline void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}
__device__ inline double buf_ld64(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline double2 buf_ld128(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
template <typename T>
__device__ inline T buf_ldT(__amdgpu_buffer_rsrc_t r, unsigned i) {
  if constexpr (sizeof(T) == 8) return buf_ld64(r, i * 8u);
  else return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(i * 4u), 0, 0));
}

}  // namespace
}  // namespace gsis
