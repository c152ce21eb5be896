// Shared device/host helpers of the mvpb HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MVPB_DEV __device__ __forceinline__
#define MVPB_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------------------
// Complex numbers, interleaved (re, im); cx<double> is 16-byte aligned for
// dwordx4 access.  cd = complex double, cf = complex float.
// ---------------------------------------------------------------------------
template <typename R>
struct __align__(2 * sizeof(R)) cx {
  R re, im;
};
using cd = cx<double>;
using cf = cx<float>;

template <typename R>
MVPB_HD cx<R> mkc(R r, R i) { cx<R> z; z.re = r; z.im = i; return z; }
MVPB_HD cd mk(double r, double i) { return mkc<double>(r, i); }
template <typename R>
MVPB_HD cx<R> czero() { return mkc<R>(R(0), R(0)); }
template <typename R>
MVPB_HD cx<R> operator+(cx<R> a, cx<R> b) { return mkc<R>(a.re + b.re, a.im + b.im); }
template <typename R>
MVPB_HD cx<R> operator-(cx<R> a, cx<R> b) { return mkc<R>(a.re - b.re, a.im - b.im); }
template <typename R>
MVPB_HD cx<R> operator-(cx<R> a) { return mkc<R>(-a.re, -a.im); }
template <typename R>
MVPB_HD cx<R> operator*(cx<R> a, cx<R> b) {
  return mkc<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
MVPB_HD cx<R> operator*(R s, cx<R> a) { return mkc<R>(s * a.re, s * a.im); }
template <typename R>
MVPB_HD cx<R> operator*(cx<R> a, R s) { return mkc<R>(s * a.re, s * a.im); }
template <typename R>
MVPB_HD cx<R> conj(cx<R> a) { return mkc<R>(a.re, -a.im); }
template <typename R>
MVPB_HD R abs2(cx<R> a) { return a.re * a.re + a.im * a.im; }
// a + b * c
template <typename R>
MVPB_HD cx<R> cfma(cx<R> b, cx<R> c, cx<R> a) {
  return mkc<R>(fma(b.re, c.re, fma(-b.im, c.im, a.re)), fma(b.re, c.im, fma(b.im, c.re, a.im)));
}
// a + conj(b) * c
template <typename R>
MVPB_HD cx<R> cfma_cj(cx<R> b, cx<R> c, cx<R> a) {
  return mkc<R>(fma(b.re, c.re, fma(b.im, c.im, a.re)), fma(b.re, c.im, fma(-b.im, c.re, a.im)));
}
template <typename R>
MVPB_HD cx<R> cdiv(cx<R> a, cx<R> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    R r = b.im / b.re, den = b.re + b.im * r;
    return mkc<R>((a.re + a.im * r) / den, (a.im - a.re * r) / den);
  } else {
    R r = b.re / b.im, den = b.re * r + b.im;
    return mkc<R>((a.re * r + a.im) / den, (a.im * r - a.re) / den);
  }
}
// precision conversions
template <typename To, typename From>
MVPB_HD cx<To> ccast(cx<From> a) { return mkc<To>((To)a.re, (To)a.im); }

// ---------------------------------------------------------------------------
// Cross-lane exchanges of a 64-wide wavefront without LDS.  Stage S of the
// butterfly pairs every lane with one partner: S = 0: lane ^ 32 and S = 1:
// lane ^ 16 (gfx950 lane-swap instructions); S = 2: mirror within 16 lanes;
// S = 3: mirror within 8; S = 4: lane ^ 2; S = 5: lane ^ 1 (DPP).  The
// partners of stage S agree in every lane-id bit above bit 5 - S, and the
// lane with that bit set is the upper one, so a halving reduction over these
// stages leaves the same values in the same lanes as one over lane ^ (32 >> S).
// ---------------------------------------------------------------------------
template <int S>
MVPB_DEV unsigned xchg_u32(unsigned v) {
  if constexpr (S == 0) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() & 32) ? r[0] : r[1];
  } else if constexpr (S == 1) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (__lane_id() & 16) ? r[0] : r[1];
  } else {
    constexpr int ctrl = S == 2 ? 0x140 : S == 3 ? 0x141 : S == 4 ? 0x4E : 0xB1;
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, true);
  }
}
template <int S>
MVPB_DEV double xchg(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = xchg_u32<S>((unsigned)b), hi = xchg_u32<S>((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int S>
MVPB_DEV float xchg(float v) {
  return __uint_as_float(xchg_u32<S>(__float_as_uint(v)));
}
// Halving step over stage S = 0 or 1 for two values at once: lanes whose
// stage-S bit (32 >> S) is clear return a + a(partner), the others
// b(partner) + b.  One lane-swap per 32-bit word and no select: the swap
// trades the upper half-group of a with the lower half-group of b.
template <int S>
MVPB_DEV double swap_add(double a, double b) {
  static_assert(S == 0 || S == 1, "lane-swap stages only");
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32);
  const unsigned blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
  unsigned l0, l1, h0, h1;
  if constexpr (S == 0) {
    const auto rl = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
  }
  const double x0 = __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0));
  const double x1 = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
  return x0 + x1;
}
// Partner value of stage S for a complex number.
template <int S, typename R>
MVPB_DEV cx<R> xchg_c(cx<R> v) {
  return mkc<R>(xchg<S>(v.re), xchg<S>(v.im));
}

// ---------------------------------------------------------------------------
// Wavefront / block reductions (64-wide wavefronts).
// ---------------------------------------------------------------------------
template <typename T>
MVPB_DEV T wave_sum_fast(T v) {
  v += xchg<0>(v);
  v += xchg<1>(v);
  v += xchg<2>(v);
  v += xchg<3>(v);
  v += xchg<4>(v);
  v += xchg<5>(v);
  return v;
}
MVPB_DEV double wave_sum(double v) { return wave_sum_fast(v); }
MVPB_DEV float wave_sum(float v) { return wave_sum_fast(v); }
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

// Complex block sum (two values in one pass); `red` holds 2*nwaves doubles.
template <typename R>
MVPB_DEV cx<R> block_sum_c(cx<R> v, double *red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  R a = wave_sum(v.re), b = wave_sum(v.im);
  if (lane == 0) { red[2 * wid] = (double)a; red[2 * wid + 1] = (double)b; }
  __syncthreads();
  double sr = 0.0, si = 0.0;
  for (int w = 0; w < nw; ++w) { sr += red[2 * w]; si += red[2 * w + 1]; }
  __syncthreads();
  return mkc<R>((R)sr, (R)si);
}

// Global-memory accessors.  Buffers reached through a work-item table are
// generic pointers to the compiler, which then emits flat accesses; those
// also count against the LDS wait counter, so an LDS wait would drain every
// global load in flight.  Accessing them through address space 1 yields
// global loads and stores.
#define MVPB_GAS __attribute__((address_space(1)))
template <typename R>
MVPB_DEV cx<R> gld(const cx<R> *p, size_t i) {
  const MVPB_GAS cx<R> *q = (const MVPB_GAS cx<R> *)(p + i);
  return mkc<R>(q->re, q->im);
}
template <typename R>
MVPB_DEV void gst(cx<R> *p, size_t i, cx<R> v) {
  MVPB_GAS cx<R> *q = (MVPB_GAS cx<R> *)(p + i);
  q->re = v.re;
  q->im = v.im;
}
MVPB_DEV double gld(const double *p, size_t i) { return *((const MVPB_GAS double *)(p + i)); }
MVPB_DEV void gst(double *p, size_t i, double v) { *((MVPB_GAS double *)(p + i)) = v; }
MVPB_DEV int gld(const int *p, size_t i) { return *((const MVPB_GAS int *)(p + i)); }
MVPB_DEV float gld(const float *p, size_t i) { return *((const MVPB_GAS float *)(p + i)); }
MVPB_DEV void gst(int *p, size_t i, int v) { *((MVPB_GAS int *)(p + i)) = v; }

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (__syncthreads also waits for every outstanding global
// access, which defeats prefetching across the barrier).
MVPB_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Host-side launch status helper.
// ---------------------------------------------------------------------------
#define MVPB_LAUNCH_CHECK() (hipGetLastError())
