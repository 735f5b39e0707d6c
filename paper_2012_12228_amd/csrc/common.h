// Shared device helpers for the ph-FT-AFQMC slice-path kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FT_DEV __device__ __forceinline__

// ---------------------------------------------------------------- complex ---
FT_DEV double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
FT_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
FT_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
FT_DEV double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
FT_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
FT_DEV double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// a - b*c
FT_DEV double2 cfnms(double2 a, double2 b, double2 c) {
  return make_double2(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
FT_DEV double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm keeps the intermediate products in range
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
FT_DEV double2 clog(double2 a) { return make_double2(0.5 * log(cabs2(a)), atan2(a.y, a.x)); }

// element conversions used by the mixed-precision GEMMs
FT_DEV double2 to_d2(double2 a) { return a; }
FT_DEV double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
FT_DEV float2 to_f2(double2 a) { return make_float2((float)a.x, (float)a.y); }
FT_DEV float2 to_f2(float2 a) { return a; }

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { typedef double2 type; };
template <> struct cplx_of<float> { typedef float2 type; };

template <typename T> FT_DEV typename cplx_of<T>::type cvt(double2 a);
template <> FT_DEV double2 cvt<double>(double2 a) { return a; }
template <> FT_DEV float2 cvt<float>(double2 a) { return to_f2(a); }
template <typename T> FT_DEV typename cplx_of<T>::type cvt(float2 a);
template <> FT_DEV double2 cvt<double>(float2 a) { return to_d2(a); }
template <> FT_DEV float2 cvt<float>(float2 a) { return a; }

FT_DEV void store_c(double2* p, double2 v) { *p = v; }
FT_DEV void store_c(float2* p, double2 v) { *p = to_f2(v); }

// ------------------------------------------------------ block reductions ---
FT_DEV double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum for blockDim.x == 256 (4 waves); every thread gets the result.
FT_DEV double block_sum_256(double v, double* red /* >= 4 doubles of LDS */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

FT_DEV double2 block_csum_256(double2 v, double* red /* >= 8 doubles */) {
  double a = wave_sum(v.x), b = wave_sum(v.y);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { red[wid] = a; red[4 + wid] = b; }
  __syncthreads();
  double2 t = make_double2((red[0] + red[1]) + (red[2] + red[3]), (red[4] + red[5]) + (red[6] + red[7]));
  __syncthreads();
  return t;
}

// XCD-aware walker mapping: workgroups are dispatched round-robin over the 8 XCDs,
// so block b runs on XCD b % 8.  Giving every tile of a walker the same residue keeps
// that walker's operands in one XCD's L2.  Returns false for padding blocks.
FT_DEV bool xcd_walker_tile(int b, int n_walkers, int tiles_per_walker, int* w, int* t) {
  const int xcd = b & 7, j = b >> 3;
  const int wi = j / tiles_per_walker;
  *t = j - wi * tiles_per_walker;
  *w = wi * 8 + xcd;
  return *w < n_walkers;
}
FT_DEV int xcd_grid_blocks(int n_walkers, int tiles_per_walker) {
  return ((n_walkers + 7) / 8) * 8 * tiles_per_walker;
}
