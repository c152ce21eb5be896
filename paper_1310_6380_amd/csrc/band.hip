// Two-stage reduction of the Hermitian operator C(k) to real symmetric
// tridiagonal form, and the back-transform of the eigenvectors.
//
//  Stage 1 (dense -> band of half-width HB).  Per panel of HB columns:
//    he2hb_panel  Householder QR of the panel below the band, one workgroup
//                 per item with the panel rows held in registers; builds the
//                 compact-WY factor T (Q = I - V T V^H).
//    he2hb_hemm   X0 = A22 V with the trailing Hermitian matrix (lower
//                 triangle stored), plus per-row-block Gram partials V^H X0
//                 formed on the matrix cores from the accumulators.
//    he2hb_wform  W = X0 T - V (T^H V^H X0 T) / 2, and the update of the
//                 first HB columns of A22 (the next panel, its diagonal block
//                 included) by -W V^H - V W^H.
//    he2hb_her2k  the same update of the rest, A22[HB:, HB:] (lower tiles),
//                 on a look-ahead stream while the next panel is factored.
//    Together: A22 <- Q^H A22 Q.
//  Stage 2 (band -> tridiagonal), hb2st.  Bulge chasing with Householder
//    reflectors of length HB on a band copy holding 2 HB subdiagonals.  A few
//    workgroups per item, all on one XCD; each wavefront runs whole sweeps,
//    and block k of sweep i starts once sweep i-1 has finished its blocks
//    0 .. k+1, so consecutive sweeps run two blocks apart.
//  Back-transform.  The stage-2 reflectors (last sweep first), then the
//    stage-1 block reflectors (last panel first), applied to the eigenvectors
//    of the tridiagonal matrix: stage 2 by backtransform_2s_wave (a sliding
//    register window per wavefront) up to order 64 HB + 1, by
//    backtransform_2s (columns in LDS) above it; stage 1 by backtransform_s1.
#include <float.h>
#include <stdlib.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

constexpr int HB_LDB = 2 * HB + 1;   // stored subdiagonals of the band copy (0 .. 2 HB)
constexpr int BT_THREADS = 512;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// Sum D doubles (D a power of two, D <= 128) over the 64 lanes of a
// wavefront by halving exchanges over the butterfly stages of xchg.  Afterwards, for D <= 64, v[0] of lane l
// holds the total of value (l >> (6 - log2 D)); for D = 128, v[k] holds the
// total of value 2 l + k.
template <int D, int S>
MVPB_DEV void wave_reduce_step(double *v, int lane) {
  if constexpr (S < 6) {
    constexpr int o = 32 >> S;
    constexpr int cur = D >> S;
    if constexpr (cur >= 2 && S <= 1) {
      constexpr int h = cur / 2;
#pragma unroll
      for (int k = 0; k < h; ++k) v[k] = swap_add<S>(v[k], v[k + h]);
    } else if constexpr (cur >= 2) {
      constexpr int h = cur / 2;
      const bool hi = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const double snd = hi ? v[k] : v[k + h];
        const double keep = hi ? v[k + h] : v[k];
        v[k] = keep + xchg<S>(snd);
      }
    } else {
      v[0] += xchg<S>(v[0]);
    }
    wave_reduce_step<D, S + 1>(v, lane);
  }
}
template <int D>
MVPB_DEV void wave_reduce_vec(double *v, int lane) {
  wave_reduce_step<D, 0>(v, lane);
}

// Sum D doubles per thread over the whole workgroup (NW wavefronts); the
// totals land in out[0 .. D-1] (LDS).  scratch holds NW * D doubles.  Two
// barriers.
template <int D, int NW>
MVPB_DEV void block_reduce_vec(double *v, double *scratch, double *out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  wave_reduce_vec<D>(v, lane);
  if (D >= 64) {
    constexpr int per = D / 64;
#pragma unroll
    for (int k = 0; k < per; ++k) scratch[w * D + per * lane + k] = v[k];
  } else {
    constexpr int sh = 6 - ilog2(D);
    if ((lane & ((1 << sh) - 1)) == 0) scratch[w * D + (lane >> sh)] = v[0];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < D; t += NW * 64) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += scratch[q * D + t];
    out[t] = s;
  }
  __syncthreads();
}

// Householder reflector H = I - tau v v^H with H^H (alpha, x) = (beta, 0),
// beta real and v[0] = 1 (the convention of LAPACK's zlarfg).  xn2 = |x|^2
// of the part below alpha.  v[1:] = x * scale.
template <typename R>
MVPB_DEV void make_reflector(cx<R> alpha, double xn2, double &beta, cx<R> &tau, cx<R> &scale) {
  const double ar = (double)alpha.re, ai = (double)alpha.im;
  if (xn2 == 0.0 && ai == 0.0) {
    beta = ar;
    tau = czero<R>();
    scale = czero<R>();
    return;
  }
  const double nrm = sqrt(ar * ar + ai * ai + xn2);
  beta = ar >= 0.0 ? -nrm : nrm;
  const double ib = 1.0 / beta;
  tau = mkc<R>((R)((beta - ar) * ib), (R)(-ai * ib));
  // 1 / (alpha - beta); |alpha - beta| >= |beta| > 0, so no scaling is needed
  const double dr = ar - beta, id = 1.0 / (dr * dr + ai * ai);
  scale = mkc<R>((R)(dr * id), (R)(-ai * id));
}

// Guarded load without a branch: the address is clamped to element 0 (always
// valid) when ok is false and the value is replaced by zero, so that many such
// loads can be in flight at once.
// Load from a clamped address with no select on the value, for prefetches:
// the caller applies the mask where the value is used, so that the wait for
// the load is not forced at the load itself.
template <typename R>
MVPB_DEV cx<R> ld_raw(const cx<R> *p, size_t idx, bool ok) {
  return gld(p, ok ? idx : 0);
}
template <typename R>
MVPB_DEV cx<R> ld_or0(const cx<R> *p, size_t idx, bool ok) {
  const cx<R> v = gld(p, ok ? idx : 0);
  return ok ? v : czero<R>();
}

// ---------------------------------------------------------------------------
// Stage 1a.  Panel QR.  Panel p covers columns c0 = p HB .. c0+HB-1; its rows
// below the band are local rows r = 0 .. m-1 (global c0+HB+r).  Thread t of
// NT holds rows t, t+NT, ... (RPT of them) of SW = HB/RPT columns at a
// time (a sub-panel); with RPT > 1 the panel is factored in HB/SW sub-panels and the
// later columns are updated by each sub-panel's block reflector.
// Output: V (unit lower trapezoidal, strictly below its diagonal) and R (on
// and above) in place, T (upper, kq x kq) in T1[p].
// ---------------------------------------------------------------------------
template <typename R, int RPT, int SW, int NT, int LO>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 2)))
he2hb_panel(const EigItem *__restrict__ items, int p) {
  typedef cx<R> C;
  static_assert(HB % SW == 0 && SW * RPT <= 2 * HB, "sub-panel width divides the panel; registers bounded");
  constexpr int DC = 2 * SW;                   // column-step reduction size (doubles)
  constexpr int CW = SW < HB ? 16 / SW : 1;    // other columns per cross-reduction round
  constexpr int DX = 2 * SW * CW;              // cross-reduction size (doubles)
  constexpr int DMAX = DC > DX ? DC : DX;
  static_assert(DMAX <= 64, "reduction too large");
  __shared__ C rowj[2][SW];
  __shared__ double scratch[(NT / 64) * DMAX];
  __shared__ double sums[DMAX];
  __shared__ C Tm[HB][HB + 1];
  __shared__ C Sx[HB][SW];    // Sx[o][t]: o < nrem: (V_s^H B)[t][o]; o >= nrem: (V_prev^H V_s)[o - nrem][t]
  __shared__ C Sb[SW][HB];    // T_s^H V_s^H B
  __shared__ C M1[HB][SW];    // (V_prev^H V_s) T_s
  __shared__ C Ub[SW][SW + 1];   // u of each column of the sub-panel
  __shared__ C taus[SW];
  const EigItem it = items[blockIdx.x];
  const int n = it.n, c0 = p * HB, m = n - c0 - HB;
  // this launch handles the items whose panel height is in (LO, RPT NT]
  if (m <= LO || m > RPT * NT) return;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  C *__restrict__ P = (C *)it.A + (size_t)c0 * ld + (c0 + HB);
  const int tid = threadIdx.x;
  for (int e = tid; e < HB * (HB + 1); e += NT) (&Tm[0][0])[e] = czero<R>();
  __syncthreads();

  C x[RPT][SW];
  for (int cs = 0; cs < kq; cs += SW) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = tid + NT * s;
#pragma unroll
      for (int t = 0; t < SW; ++t)
        x[s][t] = ld_or0<R>(P, (size_t)(cs + t) * ld + r, r < m && cs + t < HB);
    }
    // ---- column loop of the sub-panel.  The registers rotate by one column
    // per step, so that position 0 always holds the current column j:
    // position q < SW-jj holds column j+q, position q >= SW-jj holds the
    // finished column cs+q-(SW-jj).  After SW steps the order is restored.
    for (int jj = 0; jj < SW; ++jj) {
      const int nfw = SW - jj;   // positions of the current and later columns
      if (cs + jj < kq) {        // uniform over the workgroup
        const int j = cs + jj;
        if (tid == j) {
#pragma unroll
          for (int q = 0; q < SW; ++q) rowj[jj & 1][q] = x[0][q];
        }
        // partials over rows r > j, by position q: q = 0: |P[r][j]|^2;
        // q > 0: conj(P[r][j]) x_q (x_q the column at position q: a later
        // column of the panel for q < nfw, a finished reflector after)
        double acc[DC];
#pragma unroll
        for (int q = 0; q < DC; ++q) acc[q] = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = tid + NT * s;
          if (r > j && r < m) {
            // accumulated in FP64 with one FMA per real product
            const cx<double> xj = mkc<double>((double)x[s][0].re, (double)x[s][0].im);
            acc[0] = fma(xj.re, xj.re, fma(xj.im, xj.im, acc[0]));
#pragma unroll
            for (int q = 1; q < SW; ++q) {
              const cx<double> c = cfma_cj(xj, mkc<double>((double)x[s][q].re, (double)x[s][q].im),
                                           mkc<double>(acc[2 * q], acc[2 * q + 1]));
              acc[2 * q] = c.re;
              acc[2 * q + 1] = c.im;
            }
          }
        }
        block_reduce_vec<DC, (NT / 64)>(acc, scratch, sums);
        const C *rj = rowj[jj & 1];
        const C alpha = rj[0];
        double beta;
        C tau, scale;
        make_reflector<R>(alpha, sums[0], beta, tau, scale);
        const C taub = conj(tau);
        // w_q = v^H P[:, j+q] = P[j][j+q] + conj(scale) d_q for 0 < q < nfw,
        // zero for the other positions (their update below is then exact)
        C wv[SW];
#pragma unroll
        for (int q = 0; q < SW; ++q) {
          const C d = mkc<R>((R)sums[2 * q], (R)sums[2 * q + 1]);
          wv[q] = (q >= 1 && q < nfw) ? rj[q] + conj(scale) * d : czero<R>();
        }
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = tid + NT * s;
          if (r < m && r >= j) {
            const bool diag = (r == j);
            const C vr = diag ? mkc<R>(R(1), R(0)) : x[s][0] * scale;
            const C ntv = czero<R>() - taub * vr;
#pragma unroll
            for (int q = 1; q < SW; ++q) x[s][q] = cfma(ntv, wv[q], x[s][q]);
            x[s][0] = diag ? mkc<R>((R)beta, R(0)) : vr;
          }
        }
        // for T of the sub-panel (formed after its last column):
        // u_l = v_l^H v_j = conj(V[j][l]) + scale g_l (column cs+l at position
        // nfw+l), g_l = sum over r > j of conj(V[r][l]) P[r][j]
        if (tid < jj) {
          const int q = nfw + tid;
          const C g = mkc<R>((R)sums[2 * q], (R)-sums[2 * q + 1]);
          Ub[tid][jj] = conj(rj[q]) + scale * g;
        }
        if (tid == 0) taus[jj] = tau;
      }
      // rotate by one column (also for skipped steps, to restore the order)
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const C first = x[s][0];
#pragma unroll
        for (int q = 0; q + 1 < SW; ++q) x[s][q] = x[s][q + 1];
        x[s][SW - 1] = first;
      }
    }
    // ---- T of the sub-panel: T_s[0:jj, jj] = -tau_jj T_s[0:jj, 0:jj] u_jj,
    // column by column (off the per-column critical path)
    __syncthreads();
    const int swe = min(SW, kq - cs);
    for (int jj = 0; jj < swe; ++jj) {
      if (tid < jj) {
        C a = czero<R>();
        for (int l = tid; l < jj; ++l) a = cfma(Tm[cs + tid][cs + l], Ub[l][jj], a);
        Tm[cs + tid][cs + jj] = czero<R>() - taus[jj] * a;
      }
      if (tid == 0) Tm[cs + jj][cs + jj] = taus[jj];
      __syncthreads();
    }
    // ---- write the sub-panel back
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = tid + NT * s;
      if (r < m) {
#pragma unroll
        for (int t = 0; t < SW; ++t)
          if (cs + t < HB) gst(P, (size_t)(cs + t) * ld + r, x[s][t]);
      }
    }
    if (SW < HB && (cs > 0 || cs + SW < HB)) {
      const int nrem = HB - cs - SW;   // panel columns right of the sub-panel
      const int nother = nrem + cs;    // ... plus the reflector columns left of it
      // V_s of the rows this thread holds (zero above the unit diagonal)
      for (int o0 = 0; o0 < nother; o0 += CW) {
        double acc[DX];
#pragma unroll
        for (int t = 0; t < DX; ++t) acc[t] = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = tid + NT * s;
          if (r < m && r >= cs) {
#pragma unroll
            for (int u = 0; u < CW; ++u) {
              const int o = o0 + u;
              if (o < nother) {
                const bool isB = o < nrem;
                const int col = isB ? cs + SW + o : o - nrem;
                C b = gld(P, (size_t)col * ld + r);
                if (!isB && r <= col) b = czero<R>();   // r >= cs > col: never taken
#pragma unroll
                for (int t = 0; t < SW; ++t) {
                  const C vs = (r > cs + t) ? x[s][t] : (r == cs + t ? mkc<R>(R(1), R(0)) : czero<R>());
                  const C c = isB ? cfma_cj(vs, b, czero<R>()) : cfma_cj(b, vs, czero<R>());
                  acc[2 * (u * SW + t)] += (double)c.re;
                  acc[2 * (u * SW + t) + 1] += (double)c.im;
                }
              }
            }
          }
        }
        block_reduce_vec<DX, (NT / 64)>(acc, scratch, sums);
        for (int e = tid; e < CW * SW; e += NT) {
          const int u = e / SW, t = e % SW;
          if (o0 + u < nother) Sx[o0 + u][t] = mkc<R>((R)sums[2 * e], (R)sums[2 * e + 1]);
        }
      }
      __syncthreads();
      // Sb = T_s^H (V_s^H B);  M1 = (V_prev^H V_s) T_s
      for (int e = tid; e < SW * nrem; e += NT) {
        const int t = e / nrem, u = e % nrem;
        C a = czero<R>();
        for (int l = 0; l <= t; ++l) a = cfma(conj(Tm[cs + l][cs + t]), Sx[u][l], a);
        Sb[t][u] = a;
      }
      for (int e = tid; e < cs * SW; e += NT) {
        const int q = e / SW, t = e % SW;
        C a = czero<R>();
        for (int l = 0; l <= t; ++l) a = cfma(Sx[nrem + q][l], Tm[cs + l][cs + t], a);
        M1[q][t] = a;
      }
      __syncthreads();
      // T[0:cs, cs:cs+SW] = -T[0:cs, 0:cs] M1
      for (int e = tid; e < cs * SW; e += NT) {
        const int q = e / SW, t = e % SW;
        C a = czero<R>();
        for (int l = q; l < cs; ++l) a = cfma(Tm[q][l], M1[l][t], a);
        Tm[q][cs + t] = czero<R>() - a;
      }
      // B <- B - V_s Sb  (rows >= cs)
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int r = tid + NT * s;
        if (r < m && r >= cs) {
          for (int u = 0; u < nrem; ++u) {
            const size_t bi = (size_t)(cs + SW + u) * ld + r;
            C b = gld(P, bi);
#pragma unroll
            for (int t = 0; t < SW; ++t) {
              const C vs = (r > cs + t) ? x[s][t] : (r == cs + t ? mkc<R>(R(1), R(0)) : czero<R>());
              b = b - vs * Sb[t][u];
            }
            gst(P, bi, b);
          }
        }
      }
      __syncthreads();
    }
  }
  // T of the panel (kq x kq, zero-padded to HB x HB), column-major
  C *T1 = (C *)it.T1 + (size_t)p * HB * HB;
  __syncthreads();
  for (int e = tid; e < HB * HB; e += NT) {
    const int i = e % HB, jx = e / HB;
    gst(T1, e, (i < kq && jx < kq && i <= jx) ? Tm[i][jx] : czero<R>());
  }
}

// V(r, t) of panel p: unit lower trapezoidal, stored strictly below its diagonal.
template <typename R>
MVPB_DEV cx<R> panel_v(const cx<R> *Vp, size_t ld, int r, int t, int m, int kq) {
  const bool in = r < m && t < kq;
  const cx<R> v = ld_or0<R>(Vp, (size_t)t * ld + r, in && r > t);
  return (in && r == t) ? mkc<R>(R(1), R(0)) : v;
}

// ---------------------------------------------------------------------------
// Stage 1b.  X0 = A22 V for row block rb (64 rows), with A22 = A[c0+HB:, c0+HB:]
// Hermitian (lower triangle stored).  Column blocks of 32 are staged in LDS as
// full tiles (direct, conjugate-transposed or mirrored from the stored lower
// triangle).  Threads: 64 rows x 4 column phases.  Also writes the Gram
// partial V[rb]^H X0[rb] (HB x HB) of the row block.
// ---------------------------------------------------------------------------
template <typename R>
MVPB_DEV cx<R> hemm_elem(const cx<R> *A22, size_t ld, int m, int gr, int gc) {
  // A22(gr, gc) of the Hermitian trailing matrix from its lower triangle
  const bool in = gr < m && gc < m, lower = gr >= gc;
  const size_t idx = lower ? (size_t)gc * ld + gr : (size_t)gr * ld + gc;
  cx<R> v = ld_or0<R>(A22, idx, in);
  if (!lower) v.im = -v.im;
  if (gr == gc) v.im = R(0);
  return v;
}

// Matrix-core step of the complex product: C += A B with A (16 x 4) and
// B (4 x 16) complex, as four real 16x16x4 products (FP64: v_mfma_f64;
// FP32: v_mfma_f32).  Lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// holds D[row][l%16], row = l/16 + 4v (FP64) or 4(l/16) + v (FP32).
typedef double hd4_t __attribute__((ext_vector_type(4)));
typedef float hf4_t __attribute__((ext_vector_type(4)));
template <typename R>
struct CMma;
template <>
struct CMma<double> {
  typedef hd4_t acc;
  MVPB_DEV static acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  MVPB_DEV static void step(cd a, cd b, acc &cr, acc &ci) {
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.im, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.re, ci, 0, 0, 0);
  }
  // Three-product form of the complex step (Gauss): p1 += a_re b_re,
  // p2 += a_im b_im, p3 += (a_re + a_im)(b_re + b_im); then
  // re = p1 - p2, im = p3 - p1 - p2.  Three real products instead of four.
  MVPB_DEV static void step3(cd a, cd b, acc &p1, acc &p2, acc &p3) {
    p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, p1, 0, 0, 0);
    p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.im, p2, 0, 0, 0);
    p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re + a.im, b.re + b.im, p3, 0, 0, 0);
  }
  MVPB_DEV static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct CMma<float> {
  typedef hf4_t acc;
  MVPB_DEV static acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  MVPB_DEV static void step(cf a, cf b, acc &cr, acc &ci) {
    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, b.re, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.im, b.im, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, b.im, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, b.re, ci, 0, 0, 0);
  }
  MVPB_DEV static void step3(cf a, cf b, acc &p1, acc &p2, acc &p3) {
    p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, b.re, p1, 0, 0, 0);
    p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, b.im, p2, 0, 0, 0);
    p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re + a.im, b.re + b.im, p3, 0, 0, 0);
  }
  MVPB_DEV static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Work slots of the stage-1 products, S per item, item-major.  Workgroups
// are dealt to the 8 XCDs round-robin by launch order, so workgroup b takes
// slot (b % 8) per + b / 8: each XCD works through one contiguous range of
// slots, and the operands shared by the slots of one item (V, W, X0) are
// fetched into one or two of the XCDs' L2 caches instead of all eight.  The
// mapping is a bijection for any placement; only the cache reuse depends on it.
constexpr int N_XCD = 8;
// Column-block width of the trailing-matrix product (LDS tile 64 x HEMM_TC)
constexpr int HEMM_TC = 32;
MVPB_DEV bool xcd_slot(int S, int n_items, int &item, int &slot) {
  const int total = n_items * S, per = (total + N_XCD - 1) / N_XCD;
  const int b = (int)blockIdx.x;
  const int g = (b % N_XCD) * per + b / N_XCD;
  if (g >= total) return false;
  item = g / S;
  slot = g % S;
  return true;
}
static int xcd_grid(int S, int n_items) { return N_XCD * ((n_items * S + N_XCD - 1) / N_XCD); }

// X0 for row block rb (64 rows) on the matrix cores: wavefront wv owns rows
// 16 wv .. 16 wv + 15 and all HB = 16 columns; column blocks of TC are
// staged in LDS (the next block is loaded into registers meanwhile).
template <typename R>
__global__ void __launch_bounds__(256) he2hb_hemm(const EigItem *__restrict__ items, int n_items, int S, int p) {
  typedef cx<R> C;
  typedef CMma<R> M;
  constexpr int TC = HEMM_TC;
  constexpr int PER = 64 * TC / 256;   // tile elements loaded per thread
  constexpr int VPER = TC * HB / 256;  // reflector elements loaded per thread
  static_assert(3 * PER + 2 * VPER <= 64, "element flags fit one 64-bit word");
  __shared__ C tile[TC][65];        // tile[cc][rr] = A22(rb*64 + rr, cb*TC + cc); X0 of the block at the end
  __shared__ C Vc[TC][HB + 1];      // V rows of the column block
  int item, rb;
  if (!xcd_slot(S, n_items, item, rb)) return;
  const EigItem it = items[item];
  const int n = it.n, c0 = p * HB, m = n - c0 - HB;
  if (m <= 0 || rb * 64 >= m) return;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  const C *__restrict__ A22 = (const C *)it.A + (size_t)(c0 + HB) * ld + (c0 + HB);
  const C *__restrict__ Vp = (const C *)it.A + (size_t)c0 * ld + (c0 + HB);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r0 = rb * 64;
  // Element e = tid + 256 u of a 64 x TC tile: below the row block it is read
  // down a stored column (rr fastest), right of it across (cc fastest, then
  // conjugate-transposed) so that both reads are coalesced.
  // Raw values with per-element flags (bit 0: in range, bit 1: read
  // transposed, so conjugate; bit 2: diagonal, so real), applied at the LDS
  // store so that the loads stay in flight during the products.
  // One register buffer: the loads of the next column block are in flight
  // while this one is multiplied (a second buffer gained nothing: the loop
  // head waits for every outstanding load).
  C nxA[PER], vnA[VPER];
  unsigned long long flA = 0;
  auto fetch = [&](int cb0, C (&nxt)[PER], C (&vnx)[VPER], unsigned long long &fl) {
    const bool above = cb0 >= r0 + 64;   // entirely right of the diagonal block
    fl = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      int rr, cc;
      if (above) { cc = e % TC; rr = e / TC; } else { rr = e & 63; cc = e >> 6; }
      const int gr = r0 + rr, gc = cb0 + cc;
      const bool in = gr < m && gc < m, lower = gr >= gc;
      const size_t idx = lower ? (size_t)gc * ld + gr : (size_t)gr * ld + gc;
      nxt[u] = ld_raw<R>(A22, idx, in);
      fl |= (unsigned long long)((in ? 1u : 0u) | (lower ? 0u : 2u) | (gr == gc ? 4u : 0u)) << (3 * u);
    }
#pragma unroll
    for (int u = 0; u < VPER; ++u) {
      const int e = tid + 256 * u;
      const int r = cb0 + e % TC, t = e / TC;
      const bool in = r < m && t < kq;
      vnx[u] = ld_raw<R>(Vp, (size_t)t * ld + r, in && r > t);
      fl |= (unsigned long long)((in && r > t) ? 1u : 0u) << (3 * PER + 2 * u);
      fl |= (unsigned long long)((in && r == t) ? 1u : 0u) << (3 * PER + 1 + 2 * u);
    }
  };
  auto stage = [&](int cb0, const C (&nxt)[PER], const C (&vnx)[VPER], unsigned long long fl) {
    const bool above = cb0 >= r0 + 64;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      int rr, cc;
      if (above) { cc = e % TC; rr = e / TC; } else { rr = e & 63; cc = e >> 6; }
      const unsigned f = (unsigned)(fl >> (3 * u));
      C v = nxt[u];
      if (f & 2u) v.im = -v.im;
      if (f & 4u) v.im = R(0);
      tile[cc][rr] = (f & 1u) ? v : czero<R>();
    }
#pragma unroll
    for (int u = 0; u < VPER; ++u) {
      const int e = tid + 256 * u;
      const unsigned f = (unsigned)(fl >> (3 * PER + 2 * u));
      Vc[e % TC][e / TC] = (f & 1u) ? vnx[u] : ((f & 2u) ? mkc<R>(R(1), R(0)) : czero<R>());
    }
  };
  typename M::acc p1 = M::zero(), p2 = M::zero(), p3 = M::zero();   // three-product complex steps
  const int ai = lane & 15, ak = lane >> 4;   // operand slot of this lane
  auto products = [&]() {
#pragma unroll
    for (int k0 = 0; k0 < TC; k0 += 4) {
      const C a = tile[k0 + ak][16 * wv + ai];
      const C b = Vc[k0 + ak][ai];
      M::step3(a, b, p1, p2, p3);
    }
  };
  // one block ahead: the loads of the next block are in flight during the
  // products of this one (blocks past the end are fetched from clamped
  // addresses and never used)
  fetch(0, nxA, vnA, flA);
  for (int cb0 = 0; cb0 < m; cb0 += TC) {
    stage(cb0, nxA, vnA, flA);
    lds_barrier();
    fetch(cb0 + TC, nxA, vnA, flA);
    products();
    lds_barrier();
  }
  // X0 rows of this block (a lane holds D[16 wv + M::row(lane, v)][lane % 16])
  // and the Gram partial G[i][t] = sum over the block's rows of conj(V[r][i])
  // X0[r][t] on the matrix cores: the accumulators are the B operand as they
  // stand (K = the lane's rows)
  C *X0 = (C *)it.X0;
  typename M::acc g1 = M::zero(), g2 = M::zero(), g3 = M::zero();
  C vr[4];   // loaded together, ahead of the X0 stores
#pragma unroll
  for (int v = 0; v < 4; ++v) vr[v] = panel_v<R>(Vp, ld, r0 + 16 * wv + M::row(lane, v), ai, m, kq);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = 16 * wv + M::row(lane, v);
    const C x = mkc<R>(p1[v] - p2[v], p3[v] - p1[v] - p2[v]);
    if (r0 + rr < m) gst(X0, (size_t)ai * ld + r0 + rr, x);
    M::step3(conj(vr[v]), x, g1, g2, g3);
  }
  // the four wavefronts' partials summed in LDS (the tile is free)
  static_assert(4 * HB * HB <= TC * 65, "Gram partials fit the tile buffer");
  C *Gs = &tile[0][0];   // [wave][i][t]
#pragma unroll
  for (int v = 0; v < 4; ++v)
    Gs[(wv * HB + M::row(lane, v)) * HB + ai] = mkc<R>(g1[v] - g2[v], g3[v] - g1[v] - g2[v]);
  lds_barrier();
  {
    const int i = tid % HB, tt = tid / HB;   // 256 threads = HB x HB
    const C sum = Gs[(0 * HB + i) * HB + tt] + Gs[(1 * HB + i) * HB + tt] + Gs[(2 * HB + i) * HB + tt] +
                  Gs[(3 * HB + i) * HB + tt];
    gst((C *)it.M0p + (size_t)rb * HB * HB, (size_t)i + (size_t)tt * HB, sum);
  }
}

// ---------------------------------------------------------------------------
// Stage 1c.  W = X0 T - V Y / 2 with Y = T^H (V^H X0) T, for row block rb;
// then this block's rows of the next panel's columns (the first HB columns of
// A22, its diagonal block included) get the update of panel p at once,
// A22(r, c) -= W(r) V(c)^H + V(r) W(c)^H for c < HB, r >= c, so that the
// next panel can be factored while the rest of A22 is updated.  Every
// workgroup forms W of rows 0 .. HB-1 itself for the second term.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) he2hb_wform(const EigItem *__restrict__ items, int n_items, int S, int p) {
  typedef cx<R> C;
  typedef CMma<R> M;
  typedef typename M::acc A4;
  // G holds W of rows 0 .. HB-1 once Q1 is formed
  __shared__ C G[HB][HB + 1], Tm[HB][HB + 1], Q1[HB][HB + 1], Y[HB][HB + 1], V0[HB][HB + 1];
  __shared__ C Wr[64][HB + 1];   // W of the block's rows
  int item, rb;
  if (!xcd_slot(S, n_items, item, rb)) return;
  const EigItem it = items[item];
  const int n = it.n, c0 = p * HB, m = n - c0 - HB;
  if (m <= 0 || rb * 64 >= m) return;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ai = lane & 15, ak = lane >> 4;
  const int nrb = (m + 63) / 64;
  const C *M0p = (const C *)it.M0p;
  const C *T1 = (const C *)it.T1 + (size_t)p * HB * HB;
  const C *X0 = (const C *)it.X0;
  const C *Vp = (const C *)it.A + (size_t)c0 * ld + (c0 + HB);
  C *A22 = (C *)it.A + (size_t)(c0 + HB) * ld + (c0 + HB);
  C *Wm = (C *)it.Wm;
  {
    const int i = tid % HB, jx = tid / HB;   // 256 threads = HB x HB
    // the row blocks' partials in four independent chains (loads in flight together)
    C s0 = czero<R>(), s1 = czero<R>(), s2 = czero<R>(), s3 = czero<R>();
    int b = 0;
    for (; b + 4 <= nrb; b += 4) {
      s0 = s0 + gld(M0p, (size_t)b * HB * HB + tid);
      s1 = s1 + gld(M0p, (size_t)(b + 1) * HB * HB + tid);
      s2 = s2 + gld(M0p, (size_t)(b + 2) * HB * HB + tid);
      s3 = s3 + gld(M0p, (size_t)(b + 3) * HB * HB + tid);
    }
    for (; b < nrb; ++b) s0 = s0 + gld(M0p, (size_t)b * HB * HB + tid);
    G[i][jx] = (s0 + s1) + (s2 + s3);
    Tm[i][jx] = gld(T1, tid);
    V0[i][jx] = panel_v<R>(Vp, ld, i, jx, m, kq);
  }
  __syncthreads();
  {
    const int i = tid % HB, jx = tid / HB;
    C s = czero<R>();
    for (int l = 0; l <= jx; ++l) s = cfma(G[i][l], Tm[l][jx], s);
    Q1[i][jx] = s;
  }
  __syncthreads();
  {
    const int i = tid % HB, jx = tid / HB;
    C s = czero<R>();
    for (int l = 0; l <= i; ++l) s = cfma_cj(Tm[l][i], Q1[l][jx], s);
    Y[i][jx] = s;
  }
  __syncthreads();
  // W = X0 T - V Y / 2 for 16 rows r0 .. r0+15 on the matrix cores (T is upper
  // triangular and zero-padded, so the full products are exact); a lane ends
  // with W(r0 + M::row(lane, v), ai)
  auto wrows = [&](int r0, A4 &p1, A4 &p2, A4 &p3) {
    p1 = M::zero();
    p2 = M::zero();
    p3 = M::zero();
    const int ra = r0 + ai;
#pragma unroll
    for (int k0 = 0; k0 < HB; k0 += 4) {
      const C a = ld_or0<R>(X0, (size_t)(k0 + ak) * ld + ra, ra < m);
      M::step3(a, Tm[k0 + ak][ai], p1, p2, p3);
    }
#pragma unroll
    for (int k0 = 0; k0 < HB; k0 += 4) {
      const C a = panel_v<R>(Vp, ld, ra, k0 + ak, m, kq);
      M::step3(a, R(-0.5) * Y[k0 + ak][ai], p1, p2, p3);
    }
  };
  {
    A4 p1, p2, p3;
    wrows(64 * rb + 16 * wv, p1, p2, p3);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = 16 * wv + M::row(lane, v), r = 64 * rb + rr;
      const C w = mkc<R>(p1[v] - p2[v], p3[v] - p1[v] - p2[v]);
      Wr[rr][ai] = w;
      if (r < m) gst(Wm, (size_t)ai * ld + r, w);
    }
  }
  if (wv == 0) {   // W of rows 0 .. HB-1 into G (no longer needed)
    A4 p1, p2, p3;
    wrows(0, p1, p2, p3);
#pragma unroll
    for (int v = 0; v < 4; ++v) G[M::row(lane, v)][ai] = mkc<R>(p1[v] - p2[v], p3[v] - p1[v] - p2[v]);
  }
  __syncthreads();
  // this block's rows of the next panel's columns c < kq (r >= c):
  // A22(r, c) -= sum_k W(r, k) conj(V(c, k)) + V(r, k) conj(W(c, k))
  {
    // the V entries of the products and the A22 entries this lane updates
    // (rows of this block only) are loaded together, before the products
    const int ra = 64 * rb + 16 * wv + ai;
    C vr[HB / 4], cur[4];
#pragma unroll
    for (int q = 0; q < HB / 4; ++q) vr[q] = panel_v<R>(Vp, ld, ra, 4 * q + ak, m, kq);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 64 * rb + 16 * wv + M::row(lane, v), c = ai;
      cur[v] = ld_raw<R>(A22, (size_t)c * ld + r, r < m && c < kq && r >= c);
    }
    A4 p1 = M::zero(), p2 = M::zero(), p3 = M::zero();
#pragma unroll
    for (int k0 = 0; k0 < HB; k0 += 4) M::step3(Wr[16 * wv + ai][k0 + ak], conj(V0[ai][k0 + ak]), p1, p2, p3);
#pragma unroll
    for (int k0 = 0; k0 < HB; k0 += 4) M::step3(vr[k0 / 4], conj(G[ai][k0 + ak]), p1, p2, p3);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 64 * rb + 16 * wv + M::row(lane, v), c = ai;
      if (r < m && c < kq && r >= c) {
        C x = cur[v] - mkc<R>(p1[v] - p2[v], p3[v] - p1[v] - p2[v]);
        if (r == c) x.im = R(0);
        gst(A22, (size_t)c * ld + r, x);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stage 1d.  A22 <- A22 - W V^H - V W^H on the lower 64 x 64 tiles of
// A22[HB:, HB:] (the first HB columns had it from the W formation), on the
// matrix cores.  The update D = W V^H + V W^H is Hermitian: the product is
// formed for the transposed position, Out[c][r] = D[c][r] (columns of the
// tile as the M index), so that a lane's outputs D[r][c] = conj(Out[c][r])
// sit on consecutive stored rows r.  Wavefront wv owns tile columns
// 16 wv .. 16 wv + 15 and all 64 rows.  The tile being updated is read
// before the products (upper entries of diagonal tiles are written too but
// never read).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) he2hb_her2k(const EigItem *__restrict__ items, int n_items, int S, int p) {
  typedef cx<R> C;
  typedef CMma<R> M;
  typedef typename M::acc A4;
  __shared__ C Vr[HB][65], Wr[HB][65];   // [k][i]: factor rows of the tile rows r
  int item, t;
  if (!xcd_slot(S, n_items, item, t)) return;
  const EigItem it = items[item];
  const int n = it.n, c0 = p * HB, m = n - c0 - HB;
  const int mt = m - HB;   // order of the updated part A22[HB:, HB:]; its rows are factor rows + HB
  if (mt <= 0) return;
  const int nt = (mt + 63) / 64;
  if (t >= nt * (nt + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  C *__restrict__ A22 = (C *)it.A + (size_t)(c0 + 2 * HB) * ld + (c0 + 2 * HB);
  const C *__restrict__ Vp = (const C *)it.A + (size_t)c0 * ld + (c0 + HB);
  const C *__restrict__ Wm = (const C *)it.Wm;
  const int r0 = I * 64, cc0 = J * 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ai = lane & 15, ak = lane >> 4;
  // the tile values this lane updates (rows r0 + 16 rb + ai, columns
  // cc0 + 16 wv + M::row(lane, v)) seed the accumulators of three-product
  // complex steps (p1, p2, p3 of M::step3): with p1 = -Re A, p2 = 0 and
  // p3 = Im A - Re A to start, A - conj(Out) = (p2 - p1, p3 - p1 - p2)
  A4 q1[4], q2[4], q3[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int gr = r0 + 16 * rb + ai;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gc = cc0 + 16 * wv + M::row(lane, v);
      const C x = ld_or0<R>(A22, (size_t)gc * ld + gr, gc < mt && gr < mt);
      q1[rb][v] = -x.re;
      q2[rb][v] = R(0);
      q3[rb][v] = x.im - x.re;
    }
  }
  // factor rows of the tile rows into LDS; those of the tile columns (the
  // A operand, rows cc0 + 16 wv + ai) straight into registers
  for (int e = tid; e < 64 * HB; e += 256) {
    const int i = e & 63, k = e >> 6;
    const int gr = r0 + i + HB;   // factor rows
    Vr[k][i] = panel_v<R>(Vp, ld, gr, k, m, kq);
    Wr[k][i] = ld_or0<R>(Wm, (size_t)k * ld + gr, gr < m && k < kq);
  }
  C aw[HB / 4], av[HB / 4];
  {
    const int gc = cc0 + 16 * wv + ai + HB;
#pragma unroll
    for (int k4 = 0; k4 < HB / 4; ++k4) {
      const int k = 4 * k4 + ak;
      aw[k4] = ld_or0<R>(Wm, (size_t)k * ld + gc, gc < m && k < kq);   // W[c][k]
      av[k4] = panel_v<R>(Vp, ld, gc, k, m, kq);                        // V[c][k]
    }
  }
  lds_barrier();
  // Out[c][r] = sum_k W[c][k] conj(V[r][k]) + V[c][k] conj(W[r][k]) = D[c][r]
#pragma unroll
  for (int k4 = 0; k4 < HB / 4; ++k4) {
    const int k0 = 4 * k4;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const C bv = conj(Vr[k0 + ak][16 * rb + ai]);   // conj(V[r][k])
      const C bw = conj(Wr[k0 + ak][16 * rb + ai]);   // conj(W[r][k])
      M::step3(aw[k4], bv, q1[rb], q2[rb], q3[rb]);
      M::step3(av[k4], bw, q1[rb], q2[rb], q3[rb]);
    }
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int gr = r0 + 16 * rb + ai;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gc = cc0 + 16 * wv + M::row(lane, v);
      // D[r][c] = conj(Out[c][r])
      const C o = mkc<R>(q2[rb][v] - q1[rb][v], q3[rb][v] - q1[rb][v] - q2[rb][v]);
      if (gc < mt && gr < mt) gst(A22, (size_t)gc * ld + gr, o);
    }
  }
}

// ---------------------------------------------------------------------------
// Stage 2.  Bulge chasing.  Band copy WB: element (r, c), 0 <= r - c <= 2 HB,
// at WB[c * HB_LDB + (r - c)].  Sweep i, block k covers rows
// J_k = [i+1+k HB, min(i+(k+1) HB, n-1)].  Block 0 annihilates A[J_0, i];
// block k >= 1 right-applies the previous reflector to A[J_k, J_{k-1}],
// annihilates its first column and left-applies to the rest; every block
// ends with the two-sided update of A[J_k, J_k].
// Only the lower band is stored, so block k of sweep i reads and writes rows
// J_k(i) alone; of sweep i-1 only blocks k and k+1 touch those rows.  Block k
// of sweep i therefore starts once sweep i-1 has finished its blocks 0 .. k+1,
// and consecutive sweeps run two blocks apart.
// A lane of a wavefront holds row q = lane % 16 and columns 4 g .. 4 g + 3
// (g = lane / 16) of a 16 x 16 block.
// ---------------------------------------------------------------------------
MVPB_DEV long long refl_count(int t) {
  // sum_{s=1}^{t} ceil(s / HB)
  if (t <= 0) return 0;
  const long long q = t / HB, r = t % HB;
  return (long long)HB * q * (q + 1) / 2 + r * (q + 1);
}
long long refl_total(int n) {
  const int t = n - 1;
  if (t <= 0) return 0;
  const long long q = t / HB, r = t % HB;
  return (long long)HB * q * (q + 1) / 2 + r * (q + 1);
}

template <typename R>
MVPB_DEV cx<R> shfl_c(cx<R> v, int src) {
  return mkc<R>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}
template <typename R>
MVPB_DEV cx<R> readlane_c(cx<R> v, int lane);
template <>
MVPB_DEV cx<double> readlane_c(cx<double> v, int lane) {
  const long long a = __double_as_longlong(v.re), b = __double_as_longlong(v.im);
  const int a0 = __builtin_amdgcn_readlane((int)a, lane), a1 = __builtin_amdgcn_readlane((int)(a >> 32), lane);
  const int b0 = __builtin_amdgcn_readlane((int)b, lane), b1 = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return mk(__longlong_as_double(((long long)a1 << 32) | (unsigned)a0),
            __longlong_as_double(((long long)b1 << 32) | (unsigned)b0));
}
template <>
MVPB_DEV cx<float> readlane_c(cx<float> v, int lane) {
  return mkc<float>(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.re), lane)),
                    __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.im), lane)));
}

// Cross-lane moves within a row of 16 lanes (DPP).
template <int CTRL>
MVPB_DEV double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
MVPB_DEV float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
// Sum over the 16 lanes of a row; every lane of the row gets the total.
template <typename T>
MVPB_DEV T row16_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm(1,0,3,2)
  v += dpp_mov<0x4E>(v);   // quad_perm(2,3,0,1)
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return v;
}
template <typename R>
MVPB_DEV cx<R> row16_sum_c(cx<R> v) {
  return mkc<R>(row16_sum(v.re), row16_sum(v.im));
}

static_assert(HB == 16, "the lane layout of the bulge-chasing kernel assumes HB = 16");
constexpr int CH_WAVES = 8;
// workgroups per item of the bulge chasing (more than one only while every
// workgroup of the launch can be resident at once, one per CU)
constexpr int HB2ST_MAX_WG = 4;
// Layout of the bulge-chasing reflectors of one sweep (nsteps blocks of HB
// entries, starting at its first reflector's index times HB): chunks of
// V2_CHUNK consecutive blocks, entry-major within a chunk (entry j of the
// chunk's blocks consecutive; the last chunk is narrower), so that the
// writer emits one contiguous run per chunk and a back-transform load of one
// entry by consecutive blocks reads runs of V2_CHUNK entries.
constexpr int V2_CHUNK = 8;
MVPB_HD size_t v2_index(int nsteps, int k, int j) {
  const int c = k / V2_CHUNK, wd = min(V2_CHUNK, nsteps - c * V2_CHUNK);
  return (size_t)c * V2_CHUNK * HB + (size_t)j * wd + (k % V2_CHUNK);
}
// launch control words of the bulge chasing: per-XCD slot counters, the next
// item, and the item of every group of P workgroups (per XCD)
constexpr int HB2ST_CTL_ITEM = 16, HB2ST_CTL_TABLE = 32, HB2ST_MAX_XCC = 16;
size_t hb2st_ctl_ints(int n_items) { return HB2ST_CTL_TABLE + (size_t)HB2ST_MAX_XCC * 8 * ((n_items + 7) / 8); }

// Copy the band (subdiagonals 0 .. HB) of the stage-1 result into the
// working band WB (subdiagonals HB+1 .. 2 HB zero, entries of rows >= n and
// the WB_PAD_COLS columns after the last zero: the bulge chasing never writes
// them, so its block loads read zeros there without masks) and clear the item's
// progress counters: flag[0] error, flag[1] abort, flag[2 + i] blocks done by
// sweep i.
template <typename R>
__global__ void __launch_bounds__(256) hb2st_init(const EigItem *__restrict__ items, int *ctl, int ctl_ints) {
  typedef cx<R> C;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int e = threadIdx.x; e < ctl_ints; e += 256) gst(ctl, e, e < HB2ST_CTL_TABLE ? 0 : -1);
  const EigItem it = items[blockIdx.y];
  const int n = it.n;
  const size_t ld = (size_t)n;
  const C *A = (const C *)it.A;
  C *WB = (C *)it.WB;
  const size_t total = ((size_t)n + WB_PAD_COLS) * HB_LDB;
  for (size_t e = blockIdx.x * (size_t)256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int c = (int)(e / HB_LDB), d = (int)(e % HB_LDB), r = c + d;
    const bool ok = d <= HB && r < n;
    C v = ld_or0<R>(A, (size_t)c * ld + r, ok);
    if (d == 0) v.im = R(0);
    gst(WB, e, v);
  }
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n + 2; e += gridDim.x * 256) gst(it.flag, e, 0);
}

// d, e of the tridiagonal result.
template <typename R>
__global__ void __launch_bounds__(256) hb2st_fini(const EigItem *__restrict__ items) {
  typedef cx<R> C;
  const EigItem it = items[blockIdx.y];
  const int n = it.n;
  const C *WB = (const C *)it.WB;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    gst(it.d, r, (double)gld(WB, (size_t)r * HB_LDB).re);
    if (r < n - 1) gst(it.e, r, (double)gld(WB, (size_t)r * HB_LDB + 1).re);
  }
}

// XCD (accelerator complex die) the calling workgroup runs on: the XCC_ID
// hardware register, bits 3:0.
MVPB_DEV int xcc_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & 0xF; }

// Workgroup layout of the bulge chasing: P workgroups per item, all on one
// XCD so that they share its L2.  Every workgroup reads the XCD it runs on
// (XCC_ID) and takes the next slot s of that XCD; the first workgroup of each
// group of P slots claims the next item and publishes it to the other P - 1.
// The launch has 8 K P workgroups, so any round-robin placement over the 8
// XCDs leaves whole groups on each; a group that stays incomplete makes its
// item give up (bounded waits), never share blocks across L2s.
// Sweeps are dealt out in groups of G consecutive ones: sweep i belongs to
// workgroup (i / G) % P, wavefront ((i / (G P)) G + i % G) % CH_WAVES.  The
// sweeps in flight (about n / (2 HB) of them) then span several CUs; a
// hand-over between CUs costs more than two wavefronts sharing a SIMD, so
// G = CH_WAVES is the default.  Sweeps hand over within a
// workgroup through LDS counters and between workgroups through counters in
// the shared L2: the producer waits until its stores are acknowledged (the
// L1 writes through to the L2) before it bumps the counter, and the consumer
// invalidates its L1 before reading the producer's blocks.
template <typename R>
__global__ void __launch_bounds__(CH_WAVES * 64) hb2st(const EigItem *__restrict__ items, int n_items, int P, int G,
                                                      int *ctl, long long spin_limit) {
  typedef cx<R> C;
  __shared__ int prog[CH_WAVES];
  __shared__ int abort_s;
  __shared__ int claim[2];
  // reflectors of the last V2_CHUNK blocks of each wavefront's sweep, written
  // out as one contiguous run per chunk (layout of v2_index)
  __shared__ C vstage[CH_WAVES][V2_CHUNK][HB];
  if (threadIdx.x == 0) {
    const int gmax = (int)(gridDim.x / P);   // groups an XCD can hold
    const int x = xcc_id();
    const int s = atomicAdd(ctl + x, 1);
    const int grp = s / P;
    int item = -1;
    if (grp < gmax) {
      int *entry = ctl + HB2ST_CTL_TABLE + x * gmax + grp;
      if (s % P == 0) {
        item = atomicAdd(ctl + HB2ST_CTL_ITEM, 1);
        __hip_atomic_store(entry, item, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        for (long long spins = 0; spins < spin_limit; ++spins) {
          item = __hip_atomic_load(entry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (item >= 0) break;
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    claim[0] = item;
    claim[1] = s % P;
  }
  __syncthreads();
  const int item = claim[0], a = claim[1];
  if (item < 0 || item >= n_items) return;
  const EigItem it = items[item];
  const int n = it.n;
  C *__restrict__ WB = (C *)it.WB;
  C *__restrict__ V2 = (C *)it.V2;
  C *__restrict__ tau2 = (C *)it.tau2;
  int *gflag = it.flag;
  const int tid = threadIdx.x;
  if (tid < CH_WAVES) prog[tid] = -1;
  if (tid == 0) abort_s = 0;
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63, q = lane & 15, g = lane >> 4;
  // lane parts of the block offsets from the diagonal entry (s, s): the
  // entries (s + q, s - HB + 4 g + t), (s + q, s + 4 g + t), (s + 4 g + t, s + q)
  const int oy = (HB_LDB - 1) * (4 * g - HB) + q, olo = (HB_LDB - 1) * 4 * g + q, oup = (HB_LDB - 1) * q + 4 * g;
  bool aborted = false;
  const int R_ = CH_WAVES / G, gp = G * P;
  // the wavefront that runs sweep j of this workgroup's share
  auto wave_of = [&](int j) { return ((j / gp) % R_) * G + j % G; };
  const bool report = (w % G == G - 1) && P > 1;   // sweep i+1 is in another workgroup
  for (int i = gp * (w / G) + G * a + w % G; i < n - 1 && !aborted; i += CH_WAVES * P) {
    const int nsteps = (n - 1 - i + HB - 1) / HB;
    const int nprev = (n - i + HB - 1) / HB;   // blocks of sweep i-1
    const long long roff = refl_count(n - 1) - refl_count(n - 1 - i);
    const bool cross = (w % G == 0) && (P > 1) && (i > 0);   // sweep i-1 is in another workgroup
    const int wprev = wave_of(i - 1);
    C vprev = czero<R>(), tauprev = czero<R>();
    for (int k = 0; k < nsteps; ++k) {
      if (i > 0) {
        const int nd = min(k + 2, nprev);
        long long spins = 0;
        if (!cross) {
          const int need = (i - 1) * 1024 + nd;
          while (__hip_atomic_load(&prog[wprev], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
            if (__hip_atomic_load(&abort_s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
              aborted = true;
              break;
            }
            if (++spins > spin_limit) {
              aborted = true;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        } else {
          while (__hip_atomic_load(gflag + 2 + (i - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < nd) {
            if (__hip_atomic_load(gflag + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                __hip_atomic_load(&abort_s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
              aborted = true;
              break;
            }
            if (++spins > spin_limit) {
              aborted = true;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
          // the blocks of sweep i-1 were written from another CU of this XCD:
          // drop stale L1 lines before reading them
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (aborted) {
          __hip_atomic_store(&abort_s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (lane == 0) {
            __hip_atomic_store(gflag + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gflag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          break;
        }
      }
      const int s = i + 1 + k * HB;
      const int L = min(HB, n - s);
      // entry (s + a, s + b) of the band copy, a >= b, is Ws[(HB_LDB - 1) b + a]:
      // every access of the block is a lane constant plus a multiple of t
      C *const Ws = WB + (size_t)s * HB_LDB;
      // ---- every load of the task at once: the column / block being
      // annihilated and the diagonal block D = A[J_k, J_k]
      C y[4], dq[4];
      if (k == 0) {
        const C x = gld(Ws + (q - (HB_LDB - 1)), 0);   // entry (s + q, s - 1); zero past row n - 1
#pragma unroll
        for (int t = 0; t < 4; ++t) y[t] = x;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = 4 * g + t;
          y[t] = gld(Ws + (oy + (HB_LDB - 1) * t), 0);   // entry (s + q, s - HB + c); zero past row n - 1
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = 4 * g + t;
        const bool lo = q >= c;
        // entry (s + q, s + c) below the diagonal, else (s + c, s + q) conjugated;
        // zero past row or column n - 1 (padding columns)
        const C *pd = lo ? Ws + (olo + (HB_LDB - 1) * t) : Ws + (oup + t);
        C v = gld(pd, 0);
        if (!lo) v.im = -v.im;
        dq[t] = v;
      }
      C vq, tau, x;
      if (k == 0) {
        x = y[0];
      } else {
        // (a) Y <- Y - tau_p (Y v_p) v_p^H
        C vp[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) vp[t] = shfl_c(vprev, 4 * g + t);
        C yv = czero<R>();
#pragma unroll
        for (int t = 0; t < 4; ++t) yv = cfma(y[t], vp[t], yv);
        yv = yv + xchg_c<1>(yv);
        yv = yv + xchg_c<0>(yv);
        const C ty = tauprev * yv;
#pragma unroll
        for (int t = 0; t < 4; ++t) y[t] = y[t] - ty * conj(vp[t]);
        // column 0 of Y, held by the lanes of row group 0, to every row group
        x = shfl_c(y[0], q);
      }
      // (b) reflector annihilating x[1:]
      double xn2 = (q >= 1 && q < L) ? (double)abs2(x) : 0.0;
      xn2 = row16_sum(xn2);
      const C alpha = readlane_c(x, 0);
      double beta;
      C scale;
      make_reflector<R>(alpha, xn2, beta, tau, scale);
      vq = (q == 0) ? mkc<R>(R(1), R(0)) : (q < L ? x * scale : czero<R>());
      const C betac = (q == 0) ? mkc<R>((R)beta, R(0)) : czero<R>();
      if (k == 0) {
        if (g == 0 && q < L) gst(Ws + (q - (HB_LDB - 1)), 0, betac);
      } else {
        if (g == 0) y[0] = betac;
        // (c) columns c >= 1: y <- y - conj(tau) v (v^H y)
        C vh[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) vh[t] = row16_sum_c(cfma_cj(vq, y[t], czero<R>()));
        const C tv = conj(tau) * vq;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = 4 * g + t;
          if (c >= 1) y[t] = y[t] - tv * vh[t];
        }
        if (q < L) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int c = 4 * g + t;
            gst(Ws + (oy + (HB_LDB - 1) * t), 0, y[t]);
          }
        }
      }
      // (d) two-sided update of D
      {
        C vc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) vc[t] = shfl_c(vq, 4 * g + t);
        C w0 = czero<R>();
#pragma unroll
        for (int t = 0; t < 4; ++t) w0 = cfma(dq[t], vc[t], w0);
        w0 = w0 + xchg_c<1>(w0);
        w0 = w0 + xchg_c<0>(w0);
        double vw = (double)(vq.re * w0.re + vq.im * w0.im);   // Re(conj(v_q) w0_q)
        vw = row16_sum(vw);
        const R a2 = (R)(-0.5 * (double)abs2(tau) * vw);
        const C wq = tau * w0 + a2 * vq;
        C wc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) wc[t] = shfl_c(wq, 4 * g + t);
        if (q < L) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int c = 4 * g + t;
            if (c <= q) {
              C v = dq[t] - vq * conj(wc[t]) - wq * conj(vc[t]);
              if (c == q) v.im = R(0);
              gst(Ws + (olo + (HB_LDB - 1) * t), 0, v);
            }
          }
        }
      }
      __threadfence_block();
      if (lane == 0) {
        __hip_atomic_store(&prog[w], i * 1024 + k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        // the last sweep of a group also reports to the next workgroup
        if (report) {
          // every store of this wavefront acknowledged by the shared L2
          __builtin_amdgcn_s_waitcnt(0);
          __hip_atomic_store(gflag + 2 + i, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // the reflector for the back-transform (after the release: not waited
      // for), staged until its chunk of V2_CHUNK blocks is complete
      if (g == 0) vstage[w][k % V2_CHUNK][q] = vq;
      if (k % V2_CHUNK == V2_CHUNK - 1 || k == nsteps - 1) {
        const int c = k / V2_CHUNK, wd = k % V2_CHUNK + 1;
        MVPB_GAS R *dst = (MVPB_GAS R *)(V2 + (size_t)roff * HB + (size_t)c * V2_CHUNK * HB);
        for (int e = lane; e < wd * HB; e += 64) {
          const C v = vstage[w][e % wd][e / wd];   // entry j = e / wd of block c V2_CHUNK + e % wd
          __builtin_nontemporal_store(v.re, dst + 2 * e);
          __builtin_nontemporal_store(v.im, dst + 2 * e + 1);
        }
      }
      if (lane == 0) gst(tau2, roff + k, tau);
      vprev = vq;
      tauprev = tau;
    }
  }
}

// LDS index of entry (r, c) of an n x nc block of eigenvector columns: rows
// padded to nc+1 entries and skewed by one entry every 16 rows, so that the
// rows touched by one wavefront (consecutive, or 16 apart) fall in
// different banks.
MVPB_HD int zidx(int r, int c, int nc) { return r * (nc + 1) + c + (r >> 4); }
MVPB_HD size_t zbytes(int n, int nc, size_t es) { return es * ((size_t)n * (nc + 1) + (size_t)n / 16 + 1); }

// ---------------------------------------------------------------------------
// Stage-2 back-transform for orders above 64 HB + 1.  Z (n x nc columns of
// the tridiagonal eigenvectors) in LDS; apply the stage-2 reflectors sweep by
// sweep from the last.  Output Yb (complex, n x nb, column-major) in the
// reduction precision, for the stage-1 part (backtransform_s1).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(BT_THREADS) backtransform_2s(const EigItem *__restrict__ items, int nc) {
  typedef cx<R> C;
  extern __shared__ __align__(16) unsigned char shraw[];
  C *Z = (C *)shraw;   // Z[zidx(r, c, nc)]
  __shared__ C S[HB][8], S2[HB][8], Tm[HB][HB + 1];
  const EigItem it = items[blockIdx.y];
  const int n = it.n, nb = it.nb;
  if (n - 1 <= 64 * HB) return;   // item of the wavefront kernel (backtransform_2s_wave)
  const int cbase = blockIdx.x * nc;
  if (cbase >= nb) return;
  const int ncl = min(nc, nb - cbase);
  const int tid = threadIdx.x;
  const size_t ld = (size_t)n;
  for (int e = tid; e < n * nc; e += BT_THREADS) {
    const int r = e / nc, c = e % nc;
    Z[zidx(r, c, nc)] = (c < ncl) ? mkc<R>((R)gld(it.X, (size_t)r * nb + cbase + c), R(0)) : czero<R>();
  }
  __syncthreads();
  // ---- stage 2: sweeps i = n-2 .. 0; the blocks of one sweep are disjoint.
  // Thread e owns the (block, column) pair (e / ncl, e % ncl) of every sweep;
  // the reflector of the next sweep is loaded while this one is applied.
  const C *V2 = (const C *)it.V2;
  const C *tau2 = (const C *)it.tau2;
  const long long rtot = refl_count(n - 1);
  // Branch-free (clamped addresses, values of absent blocks unused), so that
  // the loads stay in flight across the loop iterations.
  auto fetch = [&](int i, C (&vv)[HB], C &tau) {
    const int ic = max(i, 0);
    const int nsteps = (n - 1 - ic + HB - 1) / HB;
    const int k = min(tid / ncl, nsteps - 1);
    const long long r0 = rtot - refl_count(n - 1 - ic);
    const C *v = V2 + (size_t)r0 * HB;
#pragma unroll
    for (int j = 0; j < HB; ++j) vv[j] = gld(v, v2_index(nsteps, k, j));
    tau = gld(tau2, r0 + k);
  };
  // three register stages: sweep i (applied now), i-1 and i-2 (in flight)
  C va[HB], vb[HB], vc2[HB], ta = czero<R>(), tb = czero<R>(), tc = czero<R>();
#pragma unroll
  for (int j = 0; j < HB; ++j) va[j] = vb[j] = vc2[j] = czero<R>();
  fetch(n - 2, va, ta);
  fetch(n - 3, vb, tb);
  auto apply = [&](int i, const C (&vcur)[HB], C tcur) {
    const int nsteps = (n - 1 - i + HB - 1) / HB;
    const int k = tid / ncl, c = tid % ncl;
    if (k < nsteps) {
      const int s = i + 1 + k * HB;
      const int L = min(HB, n - s);
      C d0 = czero<R>(), d1 = czero<R>();
#pragma unroll
      for (int j = 0; j < HB; j += 2) {
        if (j < L) d0 = cfma_cj(vcur[j], Z[zidx(s + j, c, nc)], d0);
        if (j + 1 < L) d1 = cfma_cj(vcur[j + 1], Z[zidx(s + j + 1, c, nc)], d1);
      }
      const C td = tcur * (d0 + d1);
#pragma unroll
      for (int j = 0; j < HB; ++j)
        if (j < L) Z[zidx(s + j, c, nc)] = Z[zidx(s + j, c, nc)] - vcur[j] * td;
    }
    lds_barrier();
  };
  int i = n - 2;
  for (; i >= 2; i -= 3) {
    fetch(i - 2, vc2, tc);
    apply(i, va, ta);
    fetch(i - 3, va, ta);
    apply(i - 1, vb, tb);
    fetch(i - 4, vb, tb);
    apply(i - 2, vc2, tc);
  }
  // the remaining sweeps (at most two) are already in va, vb
  if (i >= 0) apply(i, va, ta);
  if (i >= 1) apply(i - 1, vb, tb);
  C *Y = (C *)it.Yb;
  for (int e = tid; e < n * ncl; e += BT_THREADS) {
    const int r = e % n, c = e / n;
    gst(Y, (size_t)(cbase + c) * ld + r, Z[zidx(r, c, nc)]);
  }
}

// Stage-2 back-transform with one wavefront per two eigenvector columns, for
// n - 1 <= 64 HB.  During sweep i lane k holds rows i+1+16k .. i+16+16k of the
// column (zero past n-1) in registers and applies reflector (i, k) to them;
// the blocks of one sweep are disjoint, so no lane waits for another.  Between
// sweeps the window slides up by one row: every lane hands its last row to the
// next lane (DPP wave shift) and lane 0 takes row i of the tridiagonal
// eigenvector.  The register slot of a window row rotates with the sweep
// count, so the sweep loop is unrolled 16 times to keep every index static.
// The reflectors of one sweep are stored in chunks of V2_CHUNK blocks, entry
// j of a chunk's blocks consecutive (v2_index), so that a load of entry j by
// the 64 lanes touches 8 runs of 128 bytes; they are loaded one sweep ahead,
// and the wavefronts of a workgroup are columns of one item and read the same
// reflectors (the CU's L1 serves them).
constexpr int BTW_WAVES = 4;   // wavefronts per workgroup
constexpr int BTW_COLS = 2;    // eigenvector columns per wavefront
template <typename R>
MVPB_DEV cx<R> wave_shr1_c(cx<R> v);
template <>
MVPB_DEV cx<double> wave_shr1_c(cx<double> v) {
  return mk(dpp_mov<0x138>(v.re), dpp_mov<0x138>(v.im));   // lane l <- lane l-1, lane 0 <- 0
}
template <>
MVPB_DEV cx<float> wave_shr1_c(cx<float> v) {
  return mkc<float>(dpp_mov<0x138>(v.re), dpp_mov<0x138>(v.im));
}

template <typename R>
__global__ void __launch_bounds__(BTW_WAVES * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
backtransform_2s_wave(const EigItem *__restrict__ items, int n_items, int S) {
  typedef cx<R> C;
  int item, grp;   // the S column groups of an item on one XCD: its reflectors are fetched into one L2
  if (!xcd_slot(S, n_items, item, grp)) return;
  const EigItem it = items[item];
  const int n = it.n, nb = it.nb;
  if (n - 1 > 64 * HB) return;   // item of the LDS kernel (backtransform_2s)
  const int lane = threadIdx.x & 63;
  const int cb = (grp * BTW_WAVES + (threadIdx.x >> 6)) * BTW_COLS;   // first column of the wavefront
  if (cb >= nb) return;   // whole wavefronts
  const int ncw = min(BTW_COLS, nb - cb);
  const size_t ld = (size_t)n;
  const C *V2 = (const C *)it.V2;
  const C *tau2 = (const C *)it.tau2;
  const double *X = it.X;
  C *Y = (C *)it.Yb;
  const long long rtot = refl_count(n - 1);
  const int T = n - 1;   // sweeps, applied for i = n-2 .. 0
  // reflector of sweep i for this lane's block (tau = 0 where the block is
  // absent, so that the update leaves the zero rows alone), and row i+1 of
  // the input columns (the row lane 0 takes when sweep i starts)
  auto fetch = [&](int i, C (&v)[HB], C &tau, R (&xin)[BTW_COLS]) {
    const int ic = max(i, 0);
    const int nsteps = (n - 1 - ic + HB - 1) / HB;
    const bool ok = i >= 0 && lane < nsteps;
    const long long r0 = rtot - refl_count(n - 1 - ic);
    const int kl = min(lane, nsteps - 1);
#pragma unroll
    for (int j = 0; j < HB; ++j) v[j] = gld(V2, (size_t)r0 * HB + v2_index(nsteps, kl, j));
    const C t = gld(tau2, r0 + kl);
    tau = ok ? t : czero<R>();
#pragma unroll
    for (int q = 0; q < BTW_COLS; ++q) xin[q] = (R)gld(X, (size_t)(ic + 1) * nb + cb + min(q, ncw - 1));
  };
  C w[BTW_COLS][HB];
#pragma unroll
  for (int q = 0; q < BTW_COLS; ++q)
#pragma unroll
    for (int j = 0; j < HB; ++j) w[q][j] = czero<R>();
  C va[HB], vb[HB], ta, tb;
  R xa[BTW_COLS], xb[BTW_COLS];
  fetch(T - 1, va, ta, xa);
  // one sweep; S0 = slot of logical window row 0 after the slide
  auto sweep = [&](auto S0c, const C (&v)[HB], C tau, const R (&xin)[BTW_COLS]) {
    constexpr int S0 = decltype(S0c)::value;
#pragma unroll
    for (int q = 0; q < BTW_COLS; ++q) {
      const C out = w[q][S0];              // old last row (logical 15 before the slide)
      C in = wave_shr1_c<R>(out);
      if (lane == 0) in = mkc<R>(xin[q], R(0));
      w[q][S0] = in;
    }
    C d[BTW_COLS];
#pragma unroll
    for (int q = 0; q < BTW_COLS; ++q) {
      C d0 = czero<R>(), d1 = czero<R>();
#pragma unroll
      for (int j = 0; j < HB; j += 2) {
        d0 = cfma_cj(v[j], w[q][(S0 + j) % HB], d0);
        d1 = cfma_cj(v[j + 1], w[q][(S0 + j + 1) % HB], d1);
      }
      d[q] = tau * (d0 + d1);
    }
#pragma unroll
    for (int q = 0; q < BTW_COLS; ++q)
#pragma unroll
      for (int j = 0; j < HB; ++j) w[q][(S0 + j) % HB] = w[q][(S0 + j) % HB] - v[j] * d[q];
  };
  auto finish = [&](auto S0c) {
    constexpr int S0 = decltype(S0c)::value;
#pragma unroll
    for (int q = 0; q < BTW_COLS; ++q) {
      if (q >= ncw) break;
#pragma unroll
      for (int j = 0; j < HB; ++j) {
        const int r = 1 + HB * lane + j;
        if (r < n) gst(Y, (size_t)(cb + q) * ld + r, w[q][(S0 + j) % HB]);
      }
      if (lane == 0) gst(Y, (size_t)(cb + q) * ld, mkc<R>((R)gld(X, (size_t)(cb + q)), R(0)));
    }
  };
  // sweep t (t = 0 .. T-1) is i = T-1-t; the slot of row 0 after its slide
  // is (-(t+1)) mod 16 = (15 (t+1)) mod 16.  Two register stages: the
  // reflectors of sweep t+1 load while sweep t is applied.
  for (int t0 = 0; t0 < T; t0 += HB) {
#define MVPB_BTW_STEP(u, VCUR, TCUR, XCUR, VN, TN, XN)                                   \
    {                                                                                 \
      const int t = t0 + (u);                                                         \
      if (t >= T) break;                                                              \
      fetch(T - 2 - t, VN, TN, XN);                                                   \
      sweep(std::integral_constant<int, (15 * ((u) + 1)) % HB>{}, VCUR, TCUR, XCUR);   \
      if (t == T - 1) finish(std::integral_constant<int, (15 * ((u) + 1)) % HB>{});    \
    }
    MVPB_BTW_STEP(0, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(1, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(2, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(3, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(4, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(5, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(6, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(7, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(8, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(9, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(10, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(11, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(12, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(13, vb, tb, xb, va, ta, xa)
    MVPB_BTW_STEP(14, va, ta, xa, vb, tb, xb) MVPB_BTW_STEP(15, vb, tb, xb, va, ta, xa)
#undef MVPB_BTW_STEP
  }
}

// Stage-1 part of the back-transform: Y <- Q1 Y with the block reflectors of
// the panels, last panel first; nc columns of Y per workgroup in LDS.
template <typename R>
__global__ void __launch_bounds__(BT_THREADS) backtransform_s1(const EigItem *__restrict__ items, int nc, int n_items,
                                                               int groups) {
  typedef cx<R> C;
  extern __shared__ __align__(16) unsigned char shraw[];
  C *Z = (C *)shraw;   // Z[zidx(r, c, nc)]
  __shared__ C S[HB][8], S2[HB][9], Tm[HB][HB + 1];
  int item, grp;   // the column groups of an item on one XCD: its panels are fetched into one L2
  if (!xcd_slot(groups, n_items, item, grp)) return;
  const EigItem it = items[item];
  const int n = it.n, nb = it.nb;
  const int cbase = grp * nc;
  if (cbase >= nb) return;
  const int ncl = min(nc, nb - cbase);
  const int tid = threadIdx.x;
  const size_t ld = (size_t)n;
  C *Yb = (C *)it.Yb;
  for (int e = tid; e < n * nc; e += BT_THREADS) {
    const int r = e % n, c = e / n;
    Z[zidx(r, c, nc)] = (c < ncl) ? gld(Yb, (size_t)(cbase + c) * ld + r) : czero<R>();
  }
  __syncthreads();
  // panels last to first; rows c0+HB .. n-1
  const int npan = n > HB ? (n - 1) / HB : 0;   // panels with m = n - p HB - HB > 0
  const C *A = (const C *)it.A;
  constexpr int RG = BT_THREADS / HB;          // row phases of V^H Z
  const int rg = tid % RG, tt = tid / RG;      // lanes of a wavefront: consecutive rows
  for (int p = npan - 1; p >= 0; --p) {
    const int c0 = p * HB, m = n - c0 - HB;
    const int kq = min(m, HB);
    const C *Vp = A + (size_t)c0 * ld + (c0 + HB);
    const C *T1 = (const C *)it.T1 + (size_t)p * HB * HB;
    for (int e = tid; e < HB * HB; e += BT_THREADS) Tm[e % HB][e / HB] = gld(T1, e);
    // S = V^H Z[rows]: thread (rg, tt) sums rows tt+rg, tt+rg+RG, ...
    C acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = czero<R>();
    if (tt < kq) {
      // V(r, tt) = 0 for r < tt; four rows per round, their loads issued together
      constexpr int UR = 4;
      int r = tt + rg;
      for (; r + (UR - 1) * RG < m; r += UR * RG) {
        C vl[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) vl[u] = gld(Vp, (size_t)tt * ld + r + u * RG);
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int ru = r + u * RG;
          const C v = (ru == tt) ? mkc<R>(R(1), R(0)) : vl[u];
          const C *zr = Z + zidx(c0 + HB + ru, 0, nc);
#pragma unroll
          for (int c = 0; c < 8; ++c)
            if (c < ncl) acc[c] = cfma_cj(v, zr[c], acc[c]);
        }
      }
      for (; r < m; r += RG) {
        const C vl = gld(Vp, (size_t)tt * ld + r);
        const C v = (r == tt) ? mkc<R>(R(1), R(0)) : vl;
        const C *zr = Z + zidx(c0 + HB + r, 0, nc);
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < ncl) acc[c] = cfma_cj(v, zr[c], acc[c]);
      }
    }
    static_assert(RG == 32, "the row-phase sum spans the 32 lanes of a half wavefront");
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      acc[c] = acc[c] + xchg_c<1>(acc[c]);
      acc[c] = acc[c] + xchg_c<2>(acc[c]);
      acc[c] = acc[c] + xchg_c<3>(acc[c]);
      acc[c] = acc[c] + xchg_c<4>(acc[c]);
      acc[c] = acc[c] + xchg_c<5>(acc[c]);
    }
    if (rg == 0) {
#pragma unroll
      for (int c = 0; c < 8; ++c) S[tt][c] = acc[c];
    }
    lds_barrier();
    // S2 = T S
    for (int e = tid; e < HB * 8; e += BT_THREADS) {
      const int a = e / 8, c = e % 8;
      C s2 = czero<R>();
      if (a < kq)
        for (int l = a; l < kq; ++l) s2 = cfma(Tm[a][l], S[l][c], s2);
      S2[a][c] = s2;
    }
    lds_barrier();
    // Z[rows] -= V S2: one row per thread, its V row loaded once
    for (int r = tid; r < m; r += BT_THREADS) {
      C vr[HB];
#pragma unroll
      for (int l = 0; l < HB; ++l) {
        const C vl = ld_or0<R>(Vp, (size_t)l * ld + r, l < kq && r > l);
        vr[l] = (l < kq && r == l) ? mkc<R>(R(1), R(0)) : vl;
      }
      C *zr = Z + zidx(c0 + HB + r, 0, nc);
#pragma unroll 1
      for (int c = 0; c < 8; ++c) {
        if (c < ncl) {
          C s2 = czero<R>();
#pragma unroll
          for (int l = 0; l < HB; ++l) s2 = cfma(vr[l], S2[l][c], s2);
          zr[c] = zr[c] - s2;
        }
      }
    }
    lds_barrier();
  }
  C *Y = (C *)it.Yb;
  for (int e = tid; e < n * ncl; e += BT_THREADS) {
    const int r = e % n, c = e / n;
    const C z = Z[zidx(r, c, nc)];
    gst(Y, (size_t)(cbase + c) * ld + r, z);
    if (sizeof(R) != sizeof(double)) gst(it.Y, (size_t)(cbase + c) * ld + r, ccast<double>(z));
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// The panel kernel's register blocking (RPT rows per thread) follows each
// item's own panel height, so an item's arithmetic does not depend on the
// other items of the launch: one launch per height class present, and the
// items of the other classes return at once.
// Panel height classes (LO, RPT NT]: RPT rows per thread, sub-panels of SW
// columns, NT threads.  Every wavefront repeats the per-column reductions, so
// fewer wavefronts are faster, while sub-panels (SW < 16) add cross updates:
// whole 16-column panels with two rows per thread up to m = 1024.
template <typename R, int RPT, int SW, int NT, int LO>
static void launch_panel_class(const EigItem *items, int n_items, int p, int m_lo, int m_hi, hipStream_t st) {
  constexpr int hi = RPT * NT;   // class: LO < m <= hi
  if (m_hi <= LO || m_lo > hi) return;
  hipLaunchKernelGGL((he2hb_panel<R, RPT, SW, NT, LO>), dim3(n_items), dim3(NT), 0, st, items, p);
}

// Compute units of the current device (cached per device).
constexpr int MAX_DEVICES = 64;
static int g_cu_count[MAX_DEVICES];
static int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 0;
  if (!g_cu_count[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) g_cu_count[dev] = v;
  }
  return g_cu_count[dev];
}

// Stage 1 of every part, step by step: the parts are independent sets of
// items on their own streams, so that one part's latency-bound panel overlaps
// the other's bandwidth-bound trailing update.  Within a part, panel p+1
// (whose columns the W formation of panel p has updated) is factored on the
// part's stream while the rest of the trailing matrix gets the update of
// panel p on the part's look-ahead stream; the product with the trailing
// matrix of panel p+1 waits for both.
template <typename R>
static hipError_t launch_stage1_t(const ItemPart *parts, int n_parts) {
  int steps = 0;
  for (int q = 0; q < n_parts; ++q) steps = std::max(steps, stage1_steps(parts[q].n_max));
  hipError_t e = hipSuccess;
  for (int p = 0; p < steps && e == hipSuccess; ++p) {
    for (int q = 0; q < n_parts && e == hipSuccess; ++q) {
      const ItemPart &pt = parts[q];
      const EigItem *items = pt.items;
      const int n_items = pt.n_items;
      hipStream_t st = pt.stream, sa = pt.aside;
      const int c0 = p * HB, m = pt.n_max - c0 - HB;
      if (n_items <= 0 || m <= 0) continue;
      const int m_lo = std::max(1, pt.n_min - c0 - HB);
      {
        ProfScope ps(K_PANEL, st);
        launch_panel_class<R, 2, 16, 256, 0>(items, n_items, p, m_lo, m, st);
        launch_panel_class<R, 2, 16, 512, 512>(items, n_items, p, m_lo, m, st);
        launch_panel_class<R, 4, 4, 512, 1024>(items, n_items, p, m_lo, m, st);
        launch_panel_class<R, 8, 2, 512, 2048>(items, n_items, p, m_lo, m, st);
      }
      if (p > 0) e = hipStreamWaitEvent(st, pt.ev[2 * (p - 1) + 1], 0);   // update of panel p-1 done
      if (e != hipSuccess) break;
      const int nrb = (m + 63) / 64;
      {
        ProfScope ps(K_HEMM, st);
        hipLaunchKernelGGL((he2hb_hemm<R>), dim3(xcd_grid(nrb, n_items)), dim3(256), 0, st, items, n_items, nrb, p);
      }
      {
        ProfScope ps(K_WFORM, st);
        hipLaunchKernelGGL((he2hb_wform<R>), dim3(xcd_grid(nrb, n_items)), dim3(256), 0, st, items, n_items, nrb, p);
      }
      e = hipEventRecord(pt.ev[2 * p], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(sa, pt.ev[2 * p], 0);
      if (e != hipSuccess) break;
      const int nrt = (m - HB + 63) / 64;
      if (nrt > 0) {
        ProfScope ps(K_HER2K, sa);
        const int ntile = nrt * (nrt + 1) / 2;
        hipLaunchKernelGGL((he2hb_her2k<R>), dim3(xcd_grid(ntile, n_items)), dim3(256), 0, sa, items, n_items, ntile, p);
      }
      e = hipEventRecord(pt.ev[2 * p + 1], sa);
    }
  }
  // every part's stream waits for its last update
  for (int q = 0; q < n_parts && e == hipSuccess; ++q) {
    const int ns = stage1_steps(parts[q].n_max);
    if (parts[q].n_items > 0 && ns > 0) e = hipStreamWaitEvent(parts[q].stream, parts[q].ev[2 * (ns - 1) + 1], 0);
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_stage1(const ItemPart *parts, int n_parts, bool fp32) {
  return fp32 ? launch_stage1_t<float>(parts, n_parts) : launch_stage1_t<double>(parts, n_parts);
}

// Stage 2 (bulge chasing) of all items on one stream; ctl holds
// hb2st_ctl_ints(n_items) ints.  Every workgroup of the launch must be
// resident at once when P > 1, so nothing else may run beside it.
template <typename R>
static hipError_t launch_stage2_t(const EigItem *items, int n_items, int n_max, int *ctl, const Stage2Shape &sh,
                                  hipStream_t st) {
  {
    const int nmax_items_xcd = (n_items + 7) / 8;
    const int wg_max = sh.wg_max >= 1 ? std::min(sh.wg_max, HB2ST_MAX_WG) : HB2ST_MAX_WG;
    const int P = std::max(1, std::min(wg_max, device_cus() / (8 * nmax_items_xcd)));
    const int G = (sh.group >= 1 && sh.group <= CH_WAVES && CH_WAVES % sh.group == 0) ? sh.group : CH_WAVES;
    const long long spin_limit = sh.spin_limit > 0 ? sh.spin_limit : (1ll << 24);
    const int chunks = (n_max - 1 + HB - 1) / HB;
    {
      ProfScope ps(K_HB2ST_IO, st);
      hipLaunchKernelGGL((hb2st_init<R>), dim3(std::max(1, chunks), n_items), dim3(256), 0, st, items, ctl,
                         (int)hb2st_ctl_ints(n_items));
    }
    {
      ProfScope ps(K_HB2ST, st);
      hipLaunchKernelGGL((hb2st<R>), dim3(8 * nmax_items_xcd * P), dim3(CH_WAVES * 64), 0, st, items, n_items, P, G,
                         ctl, spin_limit);
    }
    {
      ProfScope ps(K_HB2ST_IO, st);
      hipLaunchKernelGGL((hb2st_fini<R>), dim3((n_max + 255) / 256, n_items), dim3(256), 0, st, items);
    }
  }
  return hipGetLastError();
}

hipError_t launch_stage2(const EigItem *items, int n_items, int n_max, bool fp32, int *ctl, const Stage2Shape &sh,
                         hipStream_t st) {
  return fp32 ? launch_stage2_t<float>(items, n_items, n_max, ctl, sh, st)
              : launch_stage2_t<double>(items, n_items, n_max, ctl, sh, st);
}

// Eigenvector columns per back-transform workgroup: bounded by the LDS
// budget, by one (block, column) pair of a stage-2 sweep per thread, and by 4
// (the stage-1 part is bound by its per-panel latency: more workgroups with
// fewer columns each finish sooner; 8 -> 4 columns: 19.88 -> 19.75 ms for the
// 60-point solve of the 2N = 882 cell).
int backtransform_cols(int n_max, bool fp32) {
  const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
  size_t cap = 1;
  while (cap < 8 && zbytes(n_max, (int)cap + 1, es) <= (size_t)BT_LDS_BYTES) ++cap;
  const size_t blocks = (size_t)std::max(1, (n_max - 1 + HB - 1) / HB);
  const size_t cap2 = (size_t)BT_THREADS / blocks;
  return (int)std::min<size_t>(4, std::max<size_t>(1, std::min(cap, cap2)));
}

hipError_t launch_backtransform(const EigItem *items, int n_items, int n_min, int n_max, int nb, bool fp32,
                                hipStream_t st) {
  ProfScope ps(K_BACKTRANSFORM, st);
  const int nc = backtransform_cols(n_max, fp32);
  const int groups = (nb + nc - 1) / nc;
  const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
  const size_t sh = zbytes(n_max, nc, es);
  // stage 2, per item: the wavefront kernel while every block of a sweep has
  // a lane (n - 1 <= 64 HB), else the LDS kernel; each skips the other's items
  const bool any_wave = n_min - 1 <= 64 * HB, any_lds = n_max - 1 > 64 * HB;
  const int gws = (nb + BTW_WAVES * BTW_COLS - 1) / (BTW_WAVES * BTW_COLS);
  const dim3 gw(xcd_grid(gws, n_items)), g1(xcd_grid(groups, n_items));
  if (fp32) {
    if (any_wave) hipLaunchKernelGGL((backtransform_2s_wave<float>), gw, dim3(BTW_WAVES * 64), 0, st, items, n_items, gws);
    if (any_lds)
      hipLaunchKernelGGL((backtransform_2s<float>), dim3(groups, n_items), dim3(BT_THREADS), sh, st, items, nc);
    hipLaunchKernelGGL((backtransform_s1<float>), g1, dim3(BT_THREADS), sh, st, items, nc, n_items, groups);
  } else {
    if (any_wave) hipLaunchKernelGGL((backtransform_2s_wave<double>), gw, dim3(BTW_WAVES * 64), 0, st, items, n_items, gws);
    if (any_lds)
      hipLaunchKernelGGL((backtransform_2s<double>), dim3(groups, n_items), dim3(BT_THREADS), sh, st, items, nc);
    hipLaunchKernelGGL((backtransform_s1<double>), g1, dim3(BT_THREADS), sh, st, items, nc, n_items, groups);
  }
  return hipGetLastError();
}

hipError_t init_band_attributes() {
  const void *fs[4] = {(const void *)backtransform_2s<double>, (const void *)backtransform_2s<float>,
                       (const void *)backtransform_s1<double>, (const void *)backtransform_s1<float>};
  for (const void *f : fs) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, BT_LDS_BYTES);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mvpb
