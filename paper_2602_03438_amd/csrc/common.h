// Shared device/host helpers of the NEGF library (complex arithmetic on double2,
// launch-error plumbing).  Complex numbers are interleaved (re, im) pairs, the
// same layout as complex128 / complex64 arrays in NumPy and torch.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace negf {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
// Native two-double vector: arrays of it indexed by unrolled loop counters stay
// in registers (arrays of HIP's double2 struct with conditional stores do not).
typedef double v2d __attribute__((ext_vector_type(2)));

__host__ __device__ inline double2 cmk(double re, double im) { double2 r; r.x = re; r.y = im; return r; }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) { return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ inline double2 cneg(double2 a) { return cmk(-a.x, -a.y); }
// 1 / a computed as conj(a) / |a|^2 with a scaling that avoids overflow of |a|^2.
__host__ __device__ inline double2 cinv(double2 a) {
  double s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  if (s == 0.0) return cmk(1.0 / 0.0, 0.0);
  double ax = a.x / s, ay = a.y / s;
  double d = (ax * ax + ay * ay) * s;
  return cmk(ax / d, -ay / d);
}

// Status codes shared with include/negf.h.
enum { ST_OK = 0, ST_EINVAL = 1, ST_ENOCONV = 2, ST_ESINGULAR = 3, ST_ENONFINITE = 4, ST_EHIP = 5, ST_ENOMEM = 6 };

}  // namespace negf
