// Assembly kernels: phase-summed structure factors on the difference grid,
// Toeplitz scatter of the compliance / density matrices, the per-cell
// coefficient combination and the per-k formation of the reduced operator.
//
// Method (arXiv:1310.6380): every entry of Phi and Omega (Sec. 4.1, eqs.
// (eo), (ep)) is an integral of a piecewise-constant weight times
// f = exp(i (K^{ab} - K^{te}) . x).  The Bloch part cancels in the
// difference, so with x = A^T H the entry depends only on the integer
// difference m = n_ab - n_te of the two plane-wave indices:
//   F_w(m, q) = sum_p w_p int_{Omega_p} exp(i 2 pi (m H1 + q H2)) dx.
// For a pixel cell this is a factored 2-D DFT
//   F_w = S o (E1 . W_w . E2^T),
// E1[m,i] = exp(i pi m (2i+1)/nx), E2[q,j] = exp(i pi q (2j+1)/ny),
// W_w[i,j] = w_{phase(i,j)}, S(m,q) = |Omega|/(nx ny) sinc(m/nx) sinc(q/ny).
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

// ---------------------------------------------------------------------------
// Structure factors, FP64 (two factored passes of the DFT contraction).
// ---------------------------------------------------------------------------

// Pass A: X[w][i][qi] = sum_j W_w[i,j] * E2[q, j], one block per pixel row i.
// wtab: [n_phases][4] weights (d11+d12, d11-d12, rho, 1).
__global__ void __launch_bounds__(256) sf_pass_a_f64(const int32_t *__restrict__ phase,
                                                     const double *__restrict__ wtab, int nx, int ny,
                                                     int M2, cd *__restrict__ X) {
  extern __shared__ double smem[];
  const int nq = 4 * M2 + 1;
  double *wl = smem;                // [4][ny]
  double *tc = wl + 4 * ny;         // cos(pi t / ny), t in [0, 2 ny)
  double *ts = tc + 2 * ny;         // sin(pi t / ny)
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    const int p = phase[i * ny + j];
#pragma unroll
    for (int w = 0; w < 4; ++w) wl[w * ny + j] = wtab[p * 4 + w];
  }
  for (int t = threadIdx.x; t < 2 * ny; t += blockDim.x) {
    double s, c;
    sincospi((double)t / (double)ny, &s, &c);
    tc[t] = c;
    ts[t] = s;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 4 * nq; idx += blockDim.x) {
    const int w = idx / nq, qi = idx % nq, q = qi - 2 * M2;
    // exact argument reduction: angle = pi * (q (2j+1) mod 2ny) / ny
    const int two_ny = 2 * ny;
    int step = ((2 * q) % two_ny + two_ny) % two_ny;
    int t = ((q % two_ny) + two_ny) % two_ny;
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < ny; ++j) {
      const double v = wl[w * ny + j];
      ar = fma(v, tc[t], ar);
      ai = fma(v, ts[t], ai);
      t += step;
      if (t >= two_ny) t -= two_ny;
    }
    X[((size_t)w * nx + i) * nq + qi] = mk(ar, ai);
  }
}

// Pass B: F[w][mi][qi] = S(m,q) * sum_i E1[m,i] X[w][i][qi]; one block per (mi, w).
__global__ void __launch_bounds__(256) sf_pass_b_f64(const cd *__restrict__ X, int nx, int ny, int M1,
                                                     int M2, double area, cd *__restrict__ F) {
  extern __shared__ double smem[];
  const int nm = 4 * M1 + 1, nq = 4 * M2 + 1;
  const int mi = blockIdx.x, w = blockIdx.y, m = mi - 2 * M1;
  double *er = smem, *ei = smem + nx;
  const int two_nx = 2 * nx;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    long t = ((long)m * (2 * i + 1)) % two_nx;
    if (t < 0) t += two_nx;
    double s, c;
    sincospi((double)t / (double)nx, &s, &c);
    er[i] = c;
    ei[i] = s;
  }
  __syncthreads();
  double sm = 1.0;
  if (m != 0) sm = sinpi((double)m / nx) / (M_PI * (double)m / nx);
  for (int qi = threadIdx.x; qi < nq; qi += blockDim.x) {
    const int q = qi - 2 * M2;
    double sq = 1.0;
    if (q != 0) sq = sinpi((double)q / ny) / (M_PI * (double)q / ny);
    cd acc = mk(0.0, 0.0);
    for (int i = 0; i < nx; ++i) acc = cfma(mk(er[i], ei[i]), X[((size_t)w * nx + i) * nq + qi], acc);
    const double s = area / ((double)nx * ny) * sm * sq;
    F[((size_t)w * nm + mi) * nq + qi] = s * acc;
  }
}

hipError_t launch_structure_factors_f64(const int32_t *phase, const double *wtab, int nx, int ny, int M1,
                                        int M2, double area, cd *X, cd *F, hipStream_t st) {
  const int nm = 4 * M1 + 1;
  ProfScope ps(K_SF, st);
  size_t sha = sizeof(double) * (4 * ny + 4 * ny);
  hipLaunchKernelGGL(sf_pass_a_f64, dim3(nx), dim3(256), sha, st, phase, wtab, nx, ny, M2, X);
  size_t shb = sizeof(double) * 2 * nx;
  hipLaunchKernelGGL(sf_pass_b_f64, dim3(nm, 4), dim3(256), shb, st, X, nx, ny, M1, M2, area, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Structure factors of a polygon cell: the subdomain integrals of
// exp(i dG.x) (Sec. 4.1, eqs. (eo), (ep)) in closed form.  By the divergence
// theorem, for dG != 0 the integral over a polygon is the sum over its
// oriented edges (midpoint m, edge vector d) of
//   (-i / |dG|^2) (dG_x d_y - dG_y d_x) exp(i dG.m) sin(dG.d / 2) / (dG.d / 2),
// and a clockwise polygon contributes minus the integral over its area, so
// holes are clockwise copies of their boundary.  dG = 2 pi T (m, q) on the
// (4 M1 + 1) x (4 M2 + 1) grid of the pixel path, F in the same layout.
// Pass 1: partial sums of one chunk of SFP_EDGES edges at 256 grid points per
// workgroup; pass 2: the chunks added in order.  FP64 throughout.
// ---------------------------------------------------------------------------
constexpr int SFP_EDGES = 256;

__global__ void __launch_bounds__(256) sf_poly_partial(const double *__restrict__ edges, const int *__restrict__ ephase,
                                                       const double *__restrict__ wtab, int n_edges, double T00,
                                                       double T01, double T10, double T11, int M1, int M2,
                                                       cd *__restrict__ P) {
  __shared__ double eg[SFP_EDGES][4];
  __shared__ double ew[SFP_EDGES][4];
  const int nq = 4 * M2 + 1, npt = (4 * M1 + 1) * nq;
  const int chunk = blockIdx.y, e0 = chunk * SFP_EDGES, ne = min(SFP_EDGES, n_edges - e0);
  for (int e = threadIdx.x; e < ne; e += 256) {
    const int ph = ephase[e0 + e];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      eg[e][k] = edges[(size_t)(e0 + e) * 4 + k];
      ew[e][k] = wtab[4 * ph + k];
    }
  }
  __syncthreads();
  const int pt = blockIdx.x * 256 + threadIdx.x;
  if (pt >= npt) return;
  const int m = pt / nq - 2 * M1, q = pt % nq - 2 * M2;
  const double gx = 2.0 * M_PI * (T00 * m + T01 * q), gy = 2.0 * M_PI * (T10 * m + T11 * q);
  cd acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = mk(0.0, 0.0);
  if (m != 0 || q != 0) {
    const double ig2 = 1.0 / (gx * gx + gy * gy);
    for (int e = 0; e < ne; ++e) {
      const double a = gx * eg[e][0] + gy * eg[e][1];
      const double u = 0.5 * (gx * eg[e][2] + gy * eg[e][3]);
      const double c = gx * eg[e][3] - gy * eg[e][2];
      double sa, ca;
      sincos(a, &sa, &ca);
      const double f = c * ig2 * (u == 0.0 ? 1.0 : sin(u) / u);
      // (-i) f (cos a + i sin a)
      const double re = f * sa, im = -f * ca;
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = acc[k] + ew[e][k] * mk(re, im);
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) P[((size_t)chunk * 4 + k) * npt + pt] = acc[k];
}

__global__ void __launch_bounds__(256) sf_poly_reduce(const cd *__restrict__ P, int n_chunks, int npt, int center,
                                                      double f00, double f01, double f02, double f03,
                                                      cd *__restrict__ F) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 4 * npt) return;
  const int k = t / npt, pt = t % npt;
  cd s = mk(0.0, 0.0);
  for (int c = 0; c < n_chunks; ++c) s = s + P[((size_t)c * 4 + k) * npt + pt];
  if (pt == center) s = mk(k == 0 ? f00 : k == 1 ? f01 : k == 2 ? f02 : f03, 0.0);
  F[(size_t)k * npt + pt] = s;
}

size_t sf_poly_scratch_bytes(int n_edges, int M1, int M2) {
  const size_t chunks = (size_t)std::max(1, (n_edges + SFP_EDGES - 1) / SFP_EDGES);
  return sizeof(cd) * chunks * 4 * (size_t)(4 * M1 + 1) * (4 * M2 + 1);
}

hipError_t launch_structure_factors_poly(const double *edges, const int *ephase, const double *wtab, int n_edges,
                                         const double T[4], const double f0[4], int M1, int M2, cd *X, cd *F,
                                         hipStream_t st) {
  ProfScope ps(K_SF, st);
  const int npt = (4 * M1 + 1) * (4 * M2 + 1);
  const int chunks = std::max(1, (n_edges + SFP_EDGES - 1) / SFP_EDGES);
  hipLaunchKernelGGL(sf_poly_partial, dim3((npt + 255) / 256, chunks), dim3(256), 0, st, edges, ephase, wtab,
                     n_edges, T[0], T[1], T[2], T[3], M1, M2, X);
  const int center = (2 * M1) * (4 * M2 + 1) + 2 * M2;
  hipLaunchKernelGGL(sf_poly_reduce, dim3((4 * npt + 255) / 256), dim3(256), 0, st, X, chunks, npt, center, f0[0],
                     f0[1], f0[2], f0[3], F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stress modes (Sec. 3: S = -Phi^-1 H* U, the stress coefficients of an
// eigenmode).  With exact integration the overlap J is |Omega| I, so
// H* = -H^T is diagonal per plane wave: V11 = -i|Omega| K1 u1,
// V22 = -i|Omega| K2 u2, V12 = -i|Omega| (K2 u1 + K1 u2), K_n = 2 pi T (Q + n)
// (Sec. 4.1 eq. (eh)).  For an isotropic cell the normal-stress block of Phi
// is [[A, B], [B, A]] with A + B = Sigma, A - B = Delta, and the shear block
// is 2 Delta (eq. (ep), d33 = 2 (d11 - d12)), so
//   S11 = -(Sigma^-1 (V11 + V22) + Delta^-1 (V11 - V22)) / 2,
//   S22 = -(Sigma^-1 (V11 + V22) - Delta^-1 (V11 - V22)) / 2,
//   S12 = -Delta^-1 V12 / 2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) stress_rhs(const cd *__restrict__ U, const double *__restrict__ Q, int nb,
                                                  int M1, int M2, double T00, double T01, double T10, double T11,
                                                  double area, cd *__restrict__ X) {
  const int N = (2 * M1 + 1) * (2 * M2 + 1);
  const int t = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;   // (r, b), r fastest
  if (e >= N * nb) return;
  const int r = e % N, b = e / N;
  const double q1 = Q[2 * t] + (double)(r / (2 * M2 + 1) - M1), q2 = Q[2 * t + 1] + (double)(r % (2 * M2 + 1) - M2);
  const double k1 = 2.0 * M_PI * (T00 * q1 + T01 * q2), k2 = 2.0 * M_PI * (T10 * q1 + T11 * q2);
  const cd *u = U + ((size_t)t * nb + b) * 2 * N;
  const cd u1 = u[r], u2 = u[N + r];
  // -i |Omega| z = |Omega| (z.im, -z.re)
  auto mi = [&](cd z) { return mk(area * z.im, -area * z.re); };
  const cd v11 = mi(k1 * u1), v22 = mi(k2 * u2), v12 = mi(k2 * u1 + k1 * u2);
  cd *x = X + (size_t)t * 3 * N * nb;
  x[(size_t)b * N + r] = v11 + v22;
  x[(size_t)N * nb + (size_t)b * N + r] = v11 - v22;
  x[(size_t)2 * N * nb + (size_t)b * N + r] = v12;
}

__global__ void __launch_bounds__(256) stress_combine(const cd *__restrict__ Z, int nb, int N, cd *__restrict__ S) {
  const int t = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= N * nb) return;
  const int r = e % N, b = e / N;
  const cd *z = Z + (size_t)t * 3 * N * nb + (size_t)b * N + r;
  const cd zs = z[0], zd = z[(size_t)N * nb], z12 = z[(size_t)2 * N * nb];
  cd *s = S + ((size_t)t * nb + b) * 3 * N;
  s[r] = -0.5 * (zs + zd);
  s[N + r] = -0.5 * (zs - zd);
  s[2 * N + r] = -0.5 * z12;
}

hipError_t launch_stress_rhs(const cd *U, const double *Q, int n_k, int nb, int M1, int M2, const double T[4],
                             double area, cd *X, hipStream_t st) {
  const int N = (2 * M1 + 1) * (2 * M2 + 1);
  hipLaunchKernelGGL(stress_rhs, dim3((N * nb + 255) / 256, n_k), dim3(256), 0, st, U, Q, nb, M1, M2, T[0], T[1],
                     T[2], T[3], area, X);
  return hipGetLastError();
}

hipError_t launch_stress_combine(const cd *Z, int n_k, int nb, int N, cd *S, hipStream_t st) {
  hipLaunchKernelGGL(stress_combine, dim3((N * nb + 255) / 256, n_k), dim3(256), 0, st, Z, nb, N, S);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Structure factors on the matrix cores.  The same factored contraction as
// above, F_w = S o (E1 . W_w . E2^T), as two real/complex GEMM passes tiled
// 16 x 16 per wavefront:
//   pass A: X_w = W_w . E2^T          (nx x ny) . (ny x nq), E2 = cos + i sin
//   pass B: F_w = S o (E1 . X_w)      (nm x nx) . (nx x nq), complex
// Precision P: 0 = FP64 inputs / FP64 accumulate (v_mfma_f64_16x16x4f64),
// 1 = FP32 inputs / FP32 accumulate (v_mfma_f32_16x16x4f32), 2 = BF16 inputs
// / FP32 accumulate (v_mfma_f32_16x16x16bf16_1k), 3 = split BF16 (three BF16
// products per product, FP32 accumulate).  Trig factors are computed
// in FP64 with exact argument reduction and rounded to the input type.
// Operand layout (16 x 16 x K): lane l supplies A[l%16][k] and B[k][l%16]
// for its K-slot, k = (l/16)*KPL + v; it receives D[row(l,v)][l%16] with
// row = 4(l/16) + v for the FP32-accumulating forms and l/16 + 4v for FP64.
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

template <int P>
struct Mma;
template <>
struct Mma<0> {
  typedef double acc;
  typedef d4_t acc4;
  static constexpr int KPL = 1;
  MVPB_DEV static acc4 zero() { return acc4{0.0, 0.0, 0.0, 0.0}; }
  MVPB_DEV static acc4 mma(const double (&a)[1], const double (&b)[1], acc4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
  MVPB_DEV static double round_in(double x) { return x; }
  // output row of register v in this lane (FP64 16x16x4: rows interleave by 4)
  MVPB_DEV static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mma<1> {
  typedef float acc;
  typedef f4_t acc4;
  static constexpr int KPL = 1;
  MVPB_DEV static acc4 zero() { return acc4{0.f, 0.f, 0.f, 0.f}; }
  MVPB_DEV static acc4 mma(const double (&a)[1], const double (&b)[1], acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[0], (float)b[0], c, 0, 0, 0);
  }
  MVPB_DEV static double round_in(double x) { return (double)(float)x; }
  MVPB_DEV static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
// round-to-nearest-even FP32 -> BF16 bits
MVPB_DEV short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
MVPB_DEV float bf16_value(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }
template <>
struct Mma<2> {
  typedef float acc;
  typedef f4_t acc4;
  static constexpr int KPL = 4;
  MVPB_DEV static acc4 zero() { return acc4{0.f, 0.f, 0.f, 0.f}; }
  MVPB_DEV static acc4 mma(const double (&a)[4], const double (&b)[4], acc4 c) {
    s4_t av, bv;
    av[0] = bf16_bits((float)a[0]); av[1] = bf16_bits((float)a[1]);
    av[2] = bf16_bits((float)a[2]); av[3] = bf16_bits((float)a[3]);
    bv[0] = bf16_bits((float)b[0]); bv[1] = bf16_bits((float)b[1]);
    bv[2] = bf16_bits((float)b[2]); bv[3] = bf16_bits((float)b[3]);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
  }
  MVPB_DEV static double round_in(double x) { return (double)bf16_value(bf16_bits((float)x)); }
  MVPB_DEV static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
// Split BF16: every FP32-rounded input x is carried as hi = bf16(x) plus
// lo = bf16(x - hi) (16 significant bits together), and each product as the
// three BF16 matrix-core products lo*hi + hi*lo + hi*hi in FP32 accumulation
// (the lo*lo term, below 2^-16 of the product, is dropped).  This is the
// three-product bfloat16 scheme of Henry, Tang and Heinecke (ARITH 2019).
template <>
struct Mma<3> {
  typedef float acc;
  typedef f4_t acc4;
  static constexpr int KPL = 4;
  MVPB_DEV static acc4 zero() { return acc4{0.f, 0.f, 0.f, 0.f}; }
  MVPB_DEV static void split(const double (&x)[4], s4_t &hi, s4_t &lo) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float f = (float)x[v];
      const short h = bf16_bits(f);
      hi[v] = h;
      lo[v] = bf16_bits(f - bf16_value(h));
    }
  }
  MVPB_DEV static acc4 mma(const double (&a)[4], const double (&b)[4], acc4 c) {
    s4_t ah, al, bh, bl;
    split(a, ah, al);
    split(b, bh, bl);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  }
  MVPB_DEV static double round_in(double x) { return (double)(float)x; }
  MVPB_DEV static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

MVPB_DEV void twiddle(long num, int n, double *c, double *s) {
  // exp(i pi num / n) with num reduced modulo 2n first
  long t = num % (2L * n);
  if (t < 0) t += 2L * n;
  sincospi((double)t / (double)n, s, c);
}

// Cells of one launch: a single cell (tables NULL) or one cell per
// blockIdx.y (device tables of phase maps, weight tables and areas).
struct SfCells {
  const int32_t *phase;
  const double *wtab;
  double area;
  const int32_t *const *phases;
  const double *const *wtabs;
  const double *areas;
  size_t xstride;   // doubles of pass scratch per cell
  size_t fstride;   // complex outputs per cell
};

// Pass A: one wavefront per (w, 16-row tile of i, 16-column tile of q).
// X is stored in FP64 as re/im planes [4][nx][nq].
template <int P>
__global__ void __launch_bounds__(256) sf_mfma_pass_a(SfCells cs, int nx, int ny, int M2, double *__restrict__ X) {
  const int32_t *__restrict__ phase = cs.phases ? cs.phases[blockIdx.y] : cs.phase;
  const double *__restrict__ wtab = cs.wtabs ? cs.wtabs[blockIdx.y] : cs.wtab;
  double *__restrict__ XR = X + blockIdx.y * cs.xstride;
  double *__restrict__ XI = XR + (size_t)4 * nx * (4 * M2 + 1);
  typedef Mma<P> T;
  constexpr int K = 4 * T::KPL;
  const int nq = 4 * M2 + 1;
  const int lane = threadIdx.x & 63;
  const int tiles_q = (nq + 15) / 16, tiles_i = (nx + 15) / 16;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= 4 * tiles_i * tiles_q) return;
  const int w = tile / (tiles_i * tiles_q);
  const int ti = (tile / tiles_q) % tiles_i, tq = tile % tiles_q;
  const int i = ti * 16 + (lane & 15);       // A row of this lane
  const int qc = tq * 16 + (lane & 15);      // B column of this lane
  const int q = qc - 2 * M2;
  typename T::acc4 accR = T::zero(), accI = T::zero();
  for (int k0 = 0; k0 < ny; k0 += K) {
    double a[T::KPL], bc[T::KPL], bs[T::KPL];
#pragma unroll
    for (int v = 0; v < T::KPL; ++v) {
      const int j = k0 + (lane >> 4) * T::KPL + v;
      a[v] = (i < nx && j < ny) ? wtab[phase[i * ny + j] * 4 + w] : 0.0;
      double c = 0.0, s = 0.0;
      if (qc < nq && j < ny) twiddle((long)q * (2 * j + 1), ny, &c, &s);
      bc[v] = c;
      bs[v] = s;
    }
    accR = T::mma(a, bc, accR);
    accI = T::mma(a, bs, accI);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int io = ti * 16 + T::row(lane, v);
    if (io < nx && qc < nq) {
      const size_t o = ((size_t)w * nx + io) * nq + qc;
      XR[o] = (double)accR[v];
      XI[o] = (double)accI[v];
    }
  }
}

// Pass B: one wavefront per (w, 16-row tile of m, 16-column tile of q).
template <int P>
__global__ void __launch_bounds__(256) sf_mfma_pass_b(SfCells cs, const double *__restrict__ X, int nx, int ny, int M1,
                                                      int M2, cd *__restrict__ Fout) {
  const double *__restrict__ XR = X + blockIdx.y * cs.xstride;
  const double *__restrict__ XI = XR + (size_t)4 * nx * (4 * M2 + 1);
  const double area = cs.areas ? cs.areas[blockIdx.y] : cs.area;
  cd *__restrict__ F = Fout + blockIdx.y * cs.fstride;
  typedef Mma<P> T;
  constexpr int K = 4 * T::KPL;
  const int nm = 4 * M1 + 1, nq = 4 * M2 + 1;
  const int lane = threadIdx.x & 63;
  const int tiles_q = (nq + 15) / 16, tiles_m = (nm + 15) / 16;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= 4 * tiles_m * tiles_q) return;
  const int w = tile / (tiles_m * tiles_q);
  const int tm = (tile / tiles_q) % tiles_m, tq = tile % tiles_q;
  const int mr = tm * 16 + (lane & 15);
  const int m = mr - 2 * M1;
  const int qc = tq * 16 + (lane & 15);
  typename T::acc4 fr = T::zero(), fi = T::zero();
  for (int k0 = 0; k0 < nx; k0 += K) {
    double ec[T::KPL], es[T::KPL], ens[T::KPL], xr[T::KPL], xi[T::KPL];
#pragma unroll
    for (int v = 0; v < T::KPL; ++v) {
      const int ii = k0 + (lane >> 4) * T::KPL + v;
      double c = 0.0, s = 0.0;
      if (mr < nm && ii < nx) twiddle((long)m * (2 * ii + 1), nx, &c, &s);
      ec[v] = c;
      es[v] = s;
      ens[v] = -s;
      const bool ok = ii < nx && qc < nq;
      const size_t o = ((size_t)w * nx + ii) * nq + qc;
      xr[v] = ok ? T::round_in(XR[o]) : 0.0;
      xi[v] = ok ? T::round_in(XI[o]) : 0.0;
    }
    fr = T::mma(ec, xr, fr);
    fr = T::mma(ens, xi, fr);
    fi = T::mma(ec, xi, fi);
    fi = T::mma(es, xr, fi);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int mo = tm * 16 + T::row(lane, v);
    if (mo < nm && qc < nq) {
      const int mm = mo - 2 * M1, qq = qc - 2 * M2;
      const double sm = (mm == 0) ? 1.0 : sinpi((double)mm / nx) / (M_PI * (double)mm / nx);
      const double sq = (qq == 0) ? 1.0 : sinpi((double)qq / ny) / (M_PI * (double)qq / ny);
      const double sc = area / ((double)nx * ny) * sm * sq;
      F[((size_t)w * nm + mo) * nq + qc] = mk(sc * (double)fr[v], sc * (double)fi[v]);
    }
  }
}

template <int P>
static void sf_mfma_launch(const SfCells &cs, int count, int nx, int ny, int M1, int M2, double *X, cd *F,
                           hipStream_t st) {
  const int nq = 4 * M2 + 1, nm = 4 * M1 + 1;
  const int ta = 4 * ((nx + 15) / 16) * ((nq + 15) / 16);
  const int tb = 4 * ((nm + 15) / 16) * ((nq + 15) / 16);
  hipLaunchKernelGGL(sf_mfma_pass_a<P>, dim3((ta + 3) / 4, count), dim3(256), 0, st, cs, nx, ny, M2, X);
  hipLaunchKernelGGL(sf_mfma_pass_b<P>, dim3((tb + 3) / 4, count), dim3(256), 0, st, cs, X, nx, ny, M1, M2, F);
}

static hipError_t sf_mfma_dispatch(int prec, const SfCells &cs, int count, int nx, int ny, int M1, int M2, double *X,
                                   cd *F, hipStream_t st) {
  ProfScope ps(K_SF, st);
  switch (prec) {
    case 0: sf_mfma_launch<0>(cs, count, nx, ny, M1, M2, X, F, st); break;
    case 1: sf_mfma_launch<1>(cs, count, nx, ny, M1, M2, X, F, st); break;
    case 3: sf_mfma_launch<3>(cs, count, nx, ny, M1, M2, X, F, st); break;
    default: sf_mfma_launch<2>(cs, count, nx, ny, M1, M2, X, F, st); break;
  }
  return hipGetLastError();
}

// X must hold 2 * 4 * nx * (4 M2 + 1) doubles.
hipError_t launch_structure_factors_mfma(int prec, const int32_t *phase, const double *wtab, int nx, int ny, int M1,
                                         int M2, double area, double *X, cd *F, hipStream_t st) {
  SfCells cs{phase, wtab, area, nullptr, nullptr, nullptr, 0, 0};
  return sf_mfma_dispatch(prec, cs, 1, nx, ny, M1, M2, X, F, st);
}

hipError_t launch_structure_factors_mfma_batch(int prec, const int32_t *const *phases, const double *const *wtabs,
                                               const double *areas, int count, int nx, int ny, int M1, int M2,
                                               double *X, cd *F, hipStream_t st) {
  const size_t xstride = (size_t)8 * nx * (4 * M2 + 1);
  const size_t fstride = (size_t)4 * (4 * M1 + 1) * (4 * M2 + 1);
  SfCells cs{nullptr, nullptr, 0.0, phases, wtabs, areas, xstride, fstride};
  return sf_mfma_dispatch(prec, cs, count, nx, ny, M1, M2, X, F, st);
}

// ---------------------------------------------------------------------------
// Toeplitz scatter: T_w[r, c] = F_w(n_c - n_r) for w = 0 (Sigma), 1 (Delta),
// 2 (rho).  Column-major N x N outputs.  n_r = (alpha_r, beta_r) with
// r = (alpha+M1)(2M2+1) + (beta+M2).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) toeplitz_scatter(const cd *__restrict__ Fin, int M1, int M2, int N,
                                                        cd *__restrict__ T0in, size_t tstride) {
  const int nb = 2 * M2 + 1, nm = 4 * M1 + 1, nq = 4 * M2 + 1;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= N) return;
  // cell blockIdx.z: its four fields and its three matrices, stored one after the other
  const cd *__restrict__ F = Fin + (size_t)blockIdx.z * 4 * nm * nq;
  cd *__restrict__ T0 = T0in + (size_t)blockIdx.z * tstride;
  cd *__restrict__ T1 = T0 + (size_t)N * N;
  cd *__restrict__ T2 = T1 + (size_t)N * N;
  const int ar = r / nb, br = r - ar * nb;
  const int ac = c / nb, bc = c - ac * nb;
  const int dm = ac - ar + 2 * M1, dq = bc - br + 2 * M2;
  const size_t o = (size_t)dm * nq + dq;
  const size_t dst = (size_t)c * N + r;
  T0[dst] = F[o];
  T1[dst] = F[(size_t)nm * nq + o];
  T2[dst] = F[(size_t)2 * nm * nq + o];
}

hipError_t launch_toeplitz_scatter(const cd *F, int M1, int M2, int N, cd *T, int count, hipStream_t st) {
  ProfScope ps(K_SCATTER, st);
  hipLaunchKernelGGL(toeplitz_scatter, dim3((N + 255) / 256, N, count), dim3(256), 0, st, F, M1, M2, N, T,
                     (size_t)3 * N * N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Combine the products X_lm = P_l P_m^H (X in {Sigma, Delta}, l, m in 0..2,
// stored at Xp[(x*9 + l*3 + m) * N*N]) into the 15 coefficient matrices of
// the reduced operator C(k) (block form; kappa = Bloch vector):
//   C11 = A11_0 + k1 A11_1 + k2 A11_2 + k1^2 S0 + k2^2 D0
//   C22 = A22_0 + k1 A22_1 + k2 A22_2 + k1^2 D0 + k2^2 S0
//   C12 = A12_0 + k1 A12_1 + k2 A12_2 + k1 k2 G0
//   C21 = A21_0 + k1 A21_1 + k2 A21_2 + k1 k2 G0
// all scaled by s = |Omega|^2 / 2.  Output order:
//   0..2 A11, 3..5 A22, 6..8 A12, 9..11 A21, 12 S0, 13 D0, 14 G0.
// ---------------------------------------------------------------------------
// blockIdx.y: cell of a batch (products 18 NN and coefficients 15 NN apart),
// its scale scales[blockIdx.y] when a table is given.
__global__ void __launch_bounds__(256) combine_coefficients(const cd *__restrict__ Xp0, size_t NN, double s0,
                                                            const double *__restrict__ scales, cd *__restrict__ coef0) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const cd *__restrict__ Xp = Xp0 + (size_t)blockIdx.y * 18 * NN;
  cd *__restrict__ coef = coef0 + (size_t)blockIdx.y * 15 * NN;
  const double s = scales ? scales[blockIdx.y] : s0;
#define S_(l, m) Xp[(size_t)(0 * 9 + (l) * 3 + (m)) * NN + e]
#define D_(l, m) Xp[(size_t)(1 * 9 + (l) * 3 + (m)) * NN + e]
  const cd s00 = S_(0, 0), s01 = S_(0, 1), s02 = S_(0, 2), s10 = S_(1, 0), s11 = S_(1, 1), s12 = S_(1, 2),
           s20 = S_(2, 0), s21 = S_(2, 1), s22 = S_(2, 2);
  const cd d00 = D_(0, 0), d01 = D_(0, 1), d02 = D_(0, 2), d10 = D_(1, 0), d11 = D_(1, 1), d12 = D_(1, 2),
           d20 = D_(2, 0), d21 = D_(2, 1), d22 = D_(2, 2);
#undef S_
#undef D_
  cd *o = coef + e;
  o[0 * NN] = s * (s11 + d11 + d22);
  o[1 * NN] = s * (s10 + s01 + d10 + d01);
  o[2 * NN] = s * (d20 + d02);
  o[3 * NN] = s * (s22 + d22 + d11);
  o[4 * NN] = s * (d10 + d01);
  o[5 * NN] = s * (s20 + s02 + d20 + d02);
  o[6 * NN] = s * (s12 - d12 + d21);
  o[7 * NN] = s * (s02 - d02 + d20);
  o[8 * NN] = s * (s10 - d10 + d01);
  o[9 * NN] = s * (s21 - d21 + d12);
  o[10 * NN] = s * (s20 - d20 + d02);
  o[11 * NN] = s * (s01 - d01 + d10);
  o[12 * NN] = s * (s00 + d00);
  o[13 * NN] = s * d00;
  o[14 * NN] = s * s00;
}

hipError_t launch_combine(const cd *Xp, int N, double s, cd *coef, hipStream_t st) {
  const size_t NN = (size_t)N * N;
  ProfScope ps(K_COMBINE, st);
  hipLaunchKernelGGL(combine_coefficients, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, Xp, NN, s,
                     (const double *)nullptr, coef);
  return hipGetLastError();
}

hipError_t launch_combine_batch(const cd *Xp, int N, const double *scales, cd *coef, int count, hipStream_t st) {
  const size_t NN = (size_t)N * N;
  ProfScope ps(K_COMBINE, st);
  hipLaunchKernelGGL(combine_coefficients, dim3((unsigned)((NN + 255) / 256), count), dim3(256), 0, st, Xp, NN, 0.0,
                     scales, coef);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-k formation of C(k) (2N x 2N, Hermitian, full storage, column-major)
// from the coefficient matrices.  One block per 32 x 32 tile (I >= J) of the
// lower triangle.  Two copies are written: the working copy, lower triangle
// only (the reduction to tridiagonal form reads and overwrites nothing
// else), and the kept copy used by the Rayleigh-Ritz step, whose upper
// triangle gets the conjugate transpose through an LDS tile, so that it is
// exactly Hermitian with a real diagonal.
// ---------------------------------------------------------------------------
// Items per workgroup of the formation: a workgroup forms one tile for
// FO_ITEMS consecutive items, its coefficient entries loaded once while the
// items share a cell (same coefficient matrices), so that the loads are paid
// once for the k points of a cell.
constexpr int FO_ITEMS = 4;

template <typename Item, typename R>
__global__ void __launch_bounds__(256) form_operator(const Item *__restrict__ items, int n_items) {
  __shared__ cd tile[32][33];
  // linear lower-triangle tile index -> (I, J), I >= J
  const int t = blockIdx.y;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int lr = threadIdx.x & 31, lc0 = threadIdx.x >> 5;
  // this thread's entries (rows I*32 + lr, columns J*32 + lc0 + 8u): the up to
  // five coefficient entries each, and whether the entry is in a mixed block
  cd a[4][5];
  bool mixed[4];
  const cd *cf_loaded = nullptr;
  int n_loaded = -1;
  for (int ii = 0; ii < FO_ITEMS; ++ii) {
    const int item = blockIdx.x * FO_ITEMS + ii;
    if (item >= n_items) break;   // uniform
    const Item it = items[item];
    if (it.dim != 0) continue;    // general layout: form_operator_general
    const int N = it.N, n = 2 * N;
    const int nt = (n + 31) / 32;
    if (t >= nt * (nt + 1) / 2) continue;
    const cd *cf = it.coef;
    if (cf != cf_loaded || N != n_loaded) {
      const size_t NN = (size_t)N * N;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = I * 32 + lr, c = J * 32 + lc0 + 8 * u;
        const bool in = r < n && c < n && r >= c;
        const int br = r >= N, bc = c >= N;
        const int i = r - br * N, j = c - bc * N;
        const size_t e = in ? (size_t)j * N + i : 0;
        // blocks (0,0), (1,1): 1, k1, k2, k1^2, k2^2; (0,1), (1,0): 1, k1, k2, k1 k2
        const int m0 = !br && !bc ? 0 : (br && bc ? 3 : (!br ? 6 : 9));
        const int m3 = !br && !bc ? 12 : (br && bc ? 13 : 14);
        const int m4 = !br && !bc ? 13 : 12;
        mixed[u] = br != bc;
        a[u][0] = cf[(size_t)m0 * NN + e];
        a[u][1] = cf[(size_t)(m0 + 1) * NN + e];
        a[u][2] = cf[(size_t)(m0 + 2) * NN + e];
        a[u][3] = cf[(size_t)m3 * NN + e];
        a[u][4] = mixed[u] ? mk(0.0, 0.0) : cf[(size_t)m4 * NN + e];
      }
      cf_loaded = cf;
      n_loaded = N;
    }
    const double k1 = it.kap1, k2 = it.kap2;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int lc = lc0 + 8 * u;
      const int r = I * 32 + lr, c = J * 32 + lc;
      cd v = mk(0.0, 0.0);
      if (r < n && c < n && r >= c) {
        if (!mixed[u])
          v = a[u][0] + k1 * a[u][1] + k2 * a[u][2] + (k1 * k1) * a[u][3] + (k2 * k2) * a[u][4];
        else
          v = a[u][0] + k1 * a[u][1] + k2 * a[u][2] + (k1 * k2) * a[u][3];
        if (r == c) v.im = 0.0;
        const size_t dst = (size_t)c * n + r;
        ((cx<R> *)it.A)[dst] = ccast<R>(v);
        it.Ak[dst] = v;
      }
      tile[lc][lr] = v;
    }
    __syncthreads();
    // mirrored tile (J, I): element (r', c') = (J*32 + lr, I*32 + lc) with r' < c'
    for (int lc = lc0; lc < 32; lc += 8) {
      const int r = J * 32 + lr, c = I * 32 + lc;
      if (r < n && c < n && r < c) it.Ak[(size_t)c * n + r] = conj(tile[lr][lc]);
    }
    __syncthreads();
  }
}

hipError_t launch_form_operator(const EigItem *items, int n_items, int n_max, bool fp32, hipStream_t st) {
  const int nt = (n_max + 31) / 32;
  const int tiles = nt * (nt + 1) / 2;
  ProfScope ps(K_FORM, st);
  if (fp32)
    hipLaunchKernelGGL((form_operator<EigItem, float>), dim3((n_items + FO_ITEMS - 1) / FO_ITEMS, tiles), dim3(256), 0,
                       st, items, n_items);
  else
    hipLaunchKernelGGL((form_operator<EigItem, double>), dim3((n_items + FO_ITEMS - 1) / FO_ITEMS, tiles), dim3(256), 0,
                       st, items, n_items);
  return hipGetLastError();
}

}  // namespace mvpb
