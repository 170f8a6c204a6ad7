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
// Sum over the 64 lanes (every lane active) by a butterfly of lane
// exchanges: each step adds the same two values on both lanes of a pair, so
// every lane ends with the same bits.
__device__ inline double wave_sum64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
// the same for a float
__device__ inline float shr1_fill(float v, float fill) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                               __builtin_bit_cast(int, v), 0x138,
                                                               0xf, 0xf, false));
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

// Workgroup barrier that orders LDS only: the fences are limited to the
// local address space, so a wave's global stores still in flight do not
// hold it at the barrier (__syncthreads waits for them).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// Row hand-over between the workgroups of a split wavefront recurrence (one
// ordinate's rows spread over parts): the producing part's top lane writes
// its value of each column with a device-scope store; an entry holds
// kHandEmpty until written, so every entry is its own ready flag and no fence
// is needed. The consuming wave takes the entries of a block of LAG steps
// (columns c0 .. c0 + LAG - 1), loaded one block ahead, polls while any is
// still empty (at most kHandSpin polls, then sets *err and waits no more),
// and puts kHandEmpty back, which leaves the buffer ready for the next launch.
constexpr unsigned long long kHandEmpty = 0x7ff4dead0000beefull;  // a signalling
                                     // NaN: no arithmetic result has this pattern
constexpr int kHandSpin = 1 << 20;

template <int LAG>
__device__ __forceinline__ void hand_take(unsigned long long *Hr, int nx, int c0,
                                          unsigned long long &hv, bool &gave_up, int32_t *err,
                                          double (&bl)[LAG]) {
  const int lane = threadIdx.x & 63;
  const int c = c0 + lane;
  const bool mine = lane < LAG && (unsigned)c < (unsigned)nx;
  // (the test sits outside the polling loop: a wait at a loop header would
  // cover every load in flight, this one only the entry's)
  if (__ballot(hv == kHandEmpty) != 0 && !gave_up) {
    for (int spin = 0;; ++spin) {   // the producing part is behind
      if (spin == kHandSpin) {
        if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        gave_up = true;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      if (mine) hv = __hip_atomic_load(Hr + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__ballot(hv == kHandEmpty) == 0) break;
    }
  }
  const double hd = __builtin_bit_cast(double, hv);
#pragma unroll
  for (int t2 = 0; t2 < LAG; ++t2) bl[t2] = rdlane(hd, t2);
  if (mine) __hip_atomic_store(Hr + c, kHandEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int cn = c + LAG;
  hv = 0;
  if (lane < LAG && (unsigned)cn < (unsigned)nx)
    hv = __hip_atomic_load(Hr + cn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the producing side: a device-scope (sc1) store, dropped at kNoCell
__device__ inline void hand_put(__amdgpu_buffer_rsrc_t Hw, double v, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), Hw, (int)off, 0, 16);
}

}  // namespace
}  // namespace gsis
