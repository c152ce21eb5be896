// Shared device/host helpers of the mvpb HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MVPB_DEV __device__ __forceinline__
#define MVPB_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// Complex double, interleaved (re, im), 16-byte aligned for dwordx4 access.
// ---------------------------------------------------------------------------
struct __align__(16) cd {
  double re, im;
};

MVPB_HD cd mk(double r, double i) { cd z; z.re = r; z.im = i; return z; }
MVPB_HD cd operator+(cd a, cd b) { return mk(a.re + b.re, a.im + b.im); }
MVPB_HD cd operator-(cd a, cd b) { return mk(a.re - b.re, a.im - b.im); }
MVPB_HD cd operator-(cd a) { return mk(-a.re, -a.im); }
MVPB_HD cd operator*(cd a, cd b) { return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
MVPB_HD cd operator*(double s, cd a) { return mk(s * a.re, s * a.im); }
MVPB_HD cd operator*(cd a, double s) { return mk(s * a.re, s * a.im); }
MVPB_HD cd conj(cd a) { return mk(a.re, -a.im); }
MVPB_HD double abs2(cd a) { return a.re * a.re + a.im * a.im; }
// a + b * c
MVPB_HD cd cfma(cd b, cd c, cd a) {
  return mk(fma(b.re, c.re, fma(-b.im, c.im, a.re)), fma(b.re, c.im, fma(b.im, c.re, a.im)));
}
// a + conj(b) * c
MVPB_HD cd cfma_cj(cd b, cd c, cd a) {
  return mk(fma(b.re, c.re, fma(b.im, c.im, a.re)), fma(b.re, c.im, fma(-b.im, c.re, a.im)));
}
MVPB_HD cd cdiv(cd a, cd b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return mk((a.re + a.im * r) / den, (a.im - a.re * r) / den);
  } else {
    double r = b.re / b.im, den = b.re * r + b.im;
    return mk((a.re * r + a.im) / den, (a.im * r - a.re) / den);
  }
}

// ---------------------------------------------------------------------------
// Wavefront / block reductions (64-wide wavefronts).
// ---------------------------------------------------------------------------
MVPB_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
MVPB_DEV int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block; `red` is LDS scratch of at least blockDim.x/64 doubles.
// Every thread receives the result.  Contains two barriers.
MVPB_DEV double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Complex block sum (two doubles in one pass); `red` holds 2*nwaves doubles.
MVPB_DEV cd block_sum_c(cd v, double *red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double a = wave_sum(v.re), b = wave_sum(v.im);
  if (lane == 0) { red[2 * wid] = a; red[2 * wid + 1] = b; }
  __syncthreads();
  cd s = mk(0.0, 0.0);
  for (int w = 0; w < nw; ++w) { s.re += red[2 * w]; s.im += red[2 * w + 1]; }
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Host-side launch status helper.
// ---------------------------------------------------------------------------
#define MVPB_LAUNCH_CHECK() (hipGetLastError())
