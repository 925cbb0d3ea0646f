// Shared device/host helpers of the mpsim HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double2 cplx;  // interleaved complex double (re, im)

#include <string>

namespace mpsim {
// Host-side extent checks of launch operands. Every device buffer of the
// library is registered (base address, bytes); while checks are switched on
// (mps_debug_check_bounds), a launcher whose operand would reach outside the
// buffer that holds its base address throws BoundsError instead of
// launching. Process-wide; off by default.
struct BoundsError {
  std::string msg;
};
void bounds_register(const void* p, size_t bytes);
// registers p unless a buffer with that base is registered; true if added
bool bounds_register_new(const void* p, size_t bytes);
void bounds_unregister(const void* p);
bool bounds_checking();
void bounds_set_checking(bool on);
// Elements lo..hi (inclusive, of `elem` bytes, relative to p) must lie in
// one registered buffer. No-op while checks are off, for p == NULL or for
// hi < lo (nothing accessed).
void bounds_require(const void* p, long lo, long hi, size_t elem, const char* what);
}  // namespace mpsim

__host__ __device__ inline cplx cmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline cplx cmulc(cplx a, cplx b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
// c ? b : a, selected per component
__host__ __device__ inline cplx csel(bool c, cplx a, cplx b) {
  return make_double2(c ? b.x : a.x, c ? b.y : a.y);
}
__host__ __device__ inline double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
// 1 / a
__host__ __device__ inline cplx cinv(cplx a) {
  double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

#define MPS_WAVE 64

// Lane exchange inside one wave through DPP row operations and the gfx950
// row-swap instructions (register moves, no LDS round trip). For bit M the
// partner of lane i is i^1 (M = 1), i^2 (M = 2), i^7 (M = 4: mirror within
// 8 lanes), i^15 (M = 8: mirror within 16 lanes), i^16 (M = 16), i^32
// (M = 32). The partner differs from i in bit M, possibly in lower bits and
// never in higher ones, which is all a butterfly reduction over bits
// M = 32, 16, ... or 1, 2, ... needs. Every lane of the wave must be active.
template <int M>
__device__ inline unsigned lane_xch_u32(unsigned v) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "lane bit");
  if constexpr (M == 1) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad [1,0,3,2]
  } else if constexpr (M == 2) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
  } else if constexpr (M == 4) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // half-row mirror
  } else if constexpr (M == 8) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row mirror
  } else if constexpr (M == 16) {
    // odd rows of the first operand trade places with even rows of the second
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (__lane_id() & 16) ? r[0] : r[1];
  } else {
    // rows 2, 3 of the first operand trade places with rows 0, 1 of the second
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() & 32) ? r[0] : r[1];
  }
}

template <int M>
__device__ inline double lane_xch(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = lane_xch_u32<M>((unsigned)b);
  const unsigned hi = lane_xch_u32<M>((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int M>
__device__ inline int lane_xch(int v) {
  return (int)lane_xch_u32<M>((unsigned)v);
}

// lane_xch for a bit that becomes a constant once the caller's loop is
// unrolled (the switch then folds away).
__device__ inline double lane_xch_bit(double v, int m) {
  switch (m) {
    case 1: return lane_xch<1>(v);
    case 2: return lane_xch<2>(v);
    case 4: return lane_xch<4>(v);
    case 8: return lane_xch<8>(v);
    case 16: return lane_xch<16>(v);
    default: return lane_xch<32>(v);
  }
}

// Sum over the 64 lanes; every lane gets the same value (each exchange adds
// the same two numbers in both lanes of a pair).
__device__ inline double wave_sum(double v) {
  v += lane_xch<1>(v);
  v += lane_xch<2>(v);
  v += lane_xch<4>(v);
  v += lane_xch<8>(v);
  v += lane_xch<16>(v);
  v += lane_xch<32>(v);
  return v;
}

// Sum over each aligned group of 8 lanes, in all 8 of them.
__device__ inline double oct_sum(double v) {
  v += lane_xch<1>(v);
  v += lane_xch<2>(v);
  v += lane_xch<4>(v);
  return v;
}

// The value of lane `src` (the same for every lane) in every lane.
__device__ inline double wave_readlane(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Lane 0's value in every lane.
__device__ inline double wave_bcast0(double v) { return wave_readlane(v, 0); }

// Block-wide sum of one double (all threads get the result). `sh` needs
// blockDim.x / 64 doubles of shared memory. Fixed reduction order.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  int nw = blockDim.x / 64;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

static inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
