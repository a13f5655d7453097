// Internal helpers shared by the libsignkrylov translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <cstdarg>
#include <cmath>

#include "signkrylov.h"

namespace sk {

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);

#define SK_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::sk::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                      __FILE__, __LINE__);                                  \
      return SK_ERR_HIP;                                                    \
    }                                                                       \
  } while (0)

#define SK_CHECK(cond, ...)          \
  do {                               \
    if (!(cond)) {                   \
      ::sk::set_error(__VA_ARGS__);  \
      return SK_ERR_ARG;             \
    }                                \
  } while (0)

#define SK_TRY(call)             \
  do {                           \
    int s_ = (call);             \
    if (s_ != SK_OK) return s_;  \
  } while (0)

// ----------------------------------------------------------------- complex
template <typename R> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };

__host__ __device__ inline double2 mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return mk(a.x * s, a.y * s); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm for a / b
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}

// loads / stores converting between storage precision and double
__device__ inline double2 ld(const double2* p) { return *p; }
__device__ inline double2 ld(const float2* p) {
  float2 v = *p;
  return mk((double)v.x, (double)v.y);
}
__device__ inline double2 cvt(double2 v) { return v; }
__device__ inline double2 cvt(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ inline void st(double2* p, double2 v) { *p = v; }
__device__ inline void st(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// ----------------------------------------------------------------- reductions
// Wave64 sum of a double (all lanes receive the result).
// Cross-lane move of a double with a DPP pattern (both 32-bit halves);
// lanes outside ROW_MASK receive 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, returned to every lane.  Register-level
// data movement (DPP) instead of LDS permutes: within quads (lane ^ 1,
// lane ^ 2), rotations by 4 and 8 within each row of 16 lanes, then row
// broadcasts 15 -> row 1, 3 and 31 -> rows 2, 3, which leave the total in
// lane 63.  The order of additions is fixed.
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);        // row_ror:4
  v += dpp_move<0x128>(v);        // row_ror:8
  v += dpp_move<0x142, 0xA>(v);   // row_bcast:15
  v += dpp_move<0x143, 0xC>(v);   // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

inline int64_t volume_of(const sk_operator* op) {
  if (!op) return 0;
  int64_t v = 1;
  for (int i = 0; i < 4; ++i) {
    if (op->dims[i] < 1) return 0;
    v *= op->dims[i];
  }
  return v;
}

int check_operator(const sk_operator* op, sk_dtype dtype);

inline size_t cbytes(sk_dtype d) { return d == SK_C128 ? 16 : 8; }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace sk
