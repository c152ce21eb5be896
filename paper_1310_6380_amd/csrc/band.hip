// Two-stage reduction of the Hermitian operator C(k) to real symmetric
// tridiagonal form, and the back-transform of the eigenvectors.
//
//  Stage 1 (dense -> band of half-width HB).  Per panel of HB columns:
//    he2hb_panel  Householder QR of the panel below the band, one workgroup
//                 per item with the panel rows held in registers; builds the
//                 compact-WY factor T (Q = I - V T V^H).
//    he2hb_hemm   X0 = A22 V with the trailing Hermitian matrix (lower
//                 triangle stored), plus per-row-block Gram partials V^H X0.
//    he2hb_wform  W = X0 T - V (T^H V^H X0 T) / 2.
//    he2hb_her2k  A22 <- A22 - W V^H - V W^H (lower tiles).
//    Together: A22 <- Q^H A22 Q.
//  Stage 2 (band -> tridiagonal), hb2st.  Bulge chasing with Householder
//    reflectors of length HB on a band copy holding 2 HB subdiagonals.  One
//    workgroup per item; each wavefront runs whole sweeps, and block k of
//    sweep i starts once sweep i-1 has finished its block k+2, so about
//    n / (3 HB) sweeps are in flight at once.
//  Back-transform, backtransform_2s.  The stage-2 reflectors (last sweep
//    first), then the stage-1 block reflectors (last panel first), applied
//    to the eigenvectors of the tridiagonal matrix held in LDS.
#include <float.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

constexpr int PQ_THREADS = 512;
constexpr int PQ_WAVES = PQ_THREADS / 64;
constexpr int HB_LDB = 2 * HB + 1;   // stored subdiagonals of the band copy (0 .. 2 HB)
constexpr int BT_THREADS = 512;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// Sum D doubles (D a power of two, D <= 128) over the 64 lanes of a
// wavefront by halving exchanges.  Afterwards, for D <= 64, v[0] of lane l
// holds the total of value (l >> (6 - log2 D)); for D = 128, v[k] holds the
// total of value 2 l + k.
template <int D, int S>
MVPB_DEV void wave_reduce_step(double *v, int lane) {
  if constexpr (S < 6) {
    constexpr int o = 32 >> S;
    constexpr int cur = D >> S;
    if constexpr (cur >= 2) {
      constexpr int h = cur / 2;
      const bool hi = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const double snd = hi ? v[k] : v[k + h];
        const double keep = hi ? v[k + h] : v[k];
        v[k] = keep + __shfl_xor(snd, o, 64);
      }
    } else {
      v[0] += __shfl_xor(v[0], o, 64);
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
  tau = mkc<R>((R)((beta - ar) / beta), (R)(-ai / beta));
  const cd s = cdiv(mk(1.0, 0.0), mk(ar - beta, ai));
  scale = ccast<R>(s);
}

// ---------------------------------------------------------------------------
// Stage 1a.  Panel QR.  Panel p covers columns c0 = p HB .. c0+HB-1; its rows
// below the band are local rows r = 0 .. m-1 (global c0+HB+r).  Thread t
// holds rows t, t+PQ_THREADS, ... (RPT of them) of SW = HB/RPT columns at a
// time (a sub-panel); with RPT > 1 the panel is factored in HB/SW sub-panels and the
// later columns are updated by each sub-panel's block reflector.
// Output: V (unit lower trapezoidal, strictly below its diagonal) and R (on
// and above) in place, T (upper, kq x kq) in T1[p].
// ---------------------------------------------------------------------------
template <typename R, int RPT>
__global__ void __launch_bounds__(PQ_THREADS) __attribute__((amdgpu_waves_per_eu(1, 2)))
he2hb_panel(const EigItem *__restrict__ items, int p) {
  typedef cx<R> C;
  constexpr int SW = HB / RPT;                 // sub-panel width held in registers
  constexpr int DC = 2 * SW;                   // column-step reduction size (doubles)
  constexpr int CW = SW < HB ? 16 / SW : 1;    // other columns per cross-reduction round
  constexpr int DX = 2 * SW * CW;              // cross-reduction size (doubles)
  constexpr int DMAX = DC > DX ? DC : DX;
  static_assert(DMAX <= 64, "reduction too large");
  __shared__ C rowj[2][SW];
  __shared__ double scratch[PQ_WAVES * DMAX];
  __shared__ double sums[DMAX];
  __shared__ C Tm[HB][HB + 1];
  __shared__ C Sx[HB][SW];    // Sx[o][t]: o < nrem: (V_s^H B)[t][o]; o >= nrem: (V_prev^H V_s)[o - nrem][t]
  __shared__ C Sb[SW][HB];    // T_s^H V_s^H B
  __shared__ C M1[HB][SW];    // (V_prev^H V_s) T_s
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N, c0 = p * HB, m = n - c0 - HB;
  // this launch handles the items whose panel height is in (RPT/2, RPT] x PQ_THREADS
  if (m <= (RPT / 2) * PQ_THREADS || m > RPT * PQ_THREADS) return;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  C *__restrict__ P = (C *)it.A + (size_t)c0 * ld + (c0 + HB);
  const int tid = threadIdx.x;
  for (int e = tid; e < HB * (HB + 1); e += PQ_THREADS) (&Tm[0][0])[e] = czero<R>();
  __syncthreads();

  C x[RPT][SW];
  for (int cs = 0; cs < kq; cs += SW) {
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = tid + PQ_THREADS * s;
#pragma unroll
      for (int t = 0; t < SW; ++t)
        x[s][t] = (r < m && cs + t < HB) ? P[(size_t)(cs + t) * ld + r] : czero<R>();
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
        // 0 < q < nfw: conj(P[r][j]) P[r][j+q]; q >= nfw: conj(V[r][l]) P[r][j]
        double acc[DC];
#pragma unroll
        for (int q = 0; q < DC; ++q) acc[q] = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = tid + PQ_THREADS * s;
          if (r > j && r < m) {
            const C xj = x[s][0];
            acc[0] += (double)(xj.re * xj.re + xj.im * xj.im);
#pragma unroll
            for (int q = 1; q < SW; ++q) {
              const C c = (q < nfw) ? cfma_cj(xj, x[s][q], czero<R>()) : cfma_cj(x[s][q], xj, czero<R>());
              acc[2 * q] += (double)c.re;
              acc[2 * q + 1] += (double)c.im;
            }
          }
        }
        block_reduce_vec<DC, PQ_WAVES>(acc, scratch, sums);
        const C *rj = rowj[jj & 1];
        const C alpha = rj[0];
        double beta;
        C tau, scale;
        make_reflector<R>(alpha, sums[0], beta, tau, scale);
        const C taub = conj(tau);
        // w_q = v^H P[:, j+q] = P[j][j+q] + conj(scale) d_q for 0 < q < nfw
        C wv[SW];
#pragma unroll
        for (int q = 0; q < SW; ++q) {
          const C d = mkc<R>((R)sums[2 * q], (R)sums[2 * q + 1]);
          wv[q] = (q >= 1 && q < nfw) ? rj[q] + conj(scale) * d : czero<R>();
        }
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
          const int r = tid + PQ_THREADS * s;
          if (r < m && r >= j) {
            const bool diag = (r == j);
            const C vr = diag ? mkc<R>(R(1), R(0)) : x[s][0] * scale;
            const C tv = taub * vr;
#pragma unroll
            for (int q = 1; q < SW; ++q)
              if (q < nfw) x[s][q] = x[s][q] - tv * wv[q];
            x[s][0] = diag ? mkc<R>((R)beta, R(0)) : vr;
          }
        }
        // T of the sub-panel, column jj: T_s[0:jj, jj] = -tau T_s[0:jj,0:jj] u,
        // u_l = v_l^H v_j = conj(V[j][l]) + scale g_l  (column cs+l at position nfw+l)
        if (tid < jj) {
          C a = czero<R>();
          for (int l = tid; l < jj; ++l) {
            const int q = nfw + l;
            const C g = mkc<R>((R)sums[2 * q], (R)sums[2 * q + 1]);
            const C u = conj(rj[q]) + scale * g;
            a = cfma(Tm[cs + tid][cs + l], u, a);
          }
          Tm[cs + tid][j] = czero<R>() - tau * a;
        }
        if (tid == 0) Tm[j][j] = tau;
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
    // ---- write the sub-panel back
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
      const int r = tid + PQ_THREADS * s;
      if (r < m) {
#pragma unroll
        for (int t = 0; t < SW; ++t)
          if (cs + t < HB) P[(size_t)(cs + t) * ld + r] = x[s][t];
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
          const int r = tid + PQ_THREADS * s;
          if (r < m && r >= cs) {
#pragma unroll
            for (int u = 0; u < CW; ++u) {
              const int o = o0 + u;
              if (o < nother) {
                const bool isB = o < nrem;
                const int col = isB ? cs + SW + o : o - nrem;
                C b = P[(size_t)col * ld + r];
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
        block_reduce_vec<DX, PQ_WAVES>(acc, scratch, sums);
        for (int e = tid; e < CW * SW; e += PQ_THREADS) {
          const int u = e / SW, t = e % SW;
          if (o0 + u < nother) Sx[o0 + u][t] = mkc<R>((R)sums[2 * e], (R)sums[2 * e + 1]);
        }
      }
      __syncthreads();
      // Sb = T_s^H (V_s^H B);  M1 = (V_prev^H V_s) T_s
      for (int e = tid; e < SW * nrem; e += PQ_THREADS) {
        const int t = e / nrem, u = e % nrem;
        C a = czero<R>();
        for (int l = 0; l <= t; ++l) a = cfma(conj(Tm[cs + l][cs + t]), Sx[u][l], a);
        Sb[t][u] = a;
      }
      for (int e = tid; e < cs * SW; e += PQ_THREADS) {
        const int q = e / SW, t = e % SW;
        C a = czero<R>();
        for (int l = 0; l <= t; ++l) a = cfma(Sx[nrem + q][l], Tm[cs + l][cs + t], a);
        M1[q][t] = a;
      }
      __syncthreads();
      // T[0:cs, cs:cs+SW] = -T[0:cs, 0:cs] M1
      for (int e = tid; e < cs * SW; e += PQ_THREADS) {
        const int q = e / SW, t = e % SW;
        C a = czero<R>();
        for (int l = q; l < cs; ++l) a = cfma(Tm[q][l], M1[l][t], a);
        Tm[q][cs + t] = czero<R>() - a;
      }
      // B <- B - V_s Sb  (rows >= cs)
#pragma unroll
      for (int s = 0; s < RPT; ++s) {
        const int r = tid + PQ_THREADS * s;
        if (r < m && r >= cs) {
          for (int u = 0; u < nrem; ++u) {
            C *bp = P + (size_t)(cs + SW + u) * ld + r;
            C b = *bp;
#pragma unroll
            for (int t = 0; t < SW; ++t) {
              const C vs = (r > cs + t) ? x[s][t] : (r == cs + t ? mkc<R>(R(1), R(0)) : czero<R>());
              b = b - vs * Sb[t][u];
            }
            *bp = b;
          }
        }
      }
      __syncthreads();
    }
  }
  // T of the panel (kq x kq, zero-padded to HB x HB), column-major
  C *T1 = (C *)it.T1 + (size_t)p * HB * HB;
  __syncthreads();
  for (int e = tid; e < HB * HB; e += PQ_THREADS) {
    const int i = e % HB, jx = e / HB;
    T1[e] = (i < kq && jx < kq && i <= jx) ? Tm[i][jx] : czero<R>();
  }
}

// V(r, t) of panel p: unit lower trapezoidal, stored strictly below its diagonal.
template <typename R>
MVPB_DEV cx<R> panel_v(const cx<R> *Vp, size_t ld, int r, int t, int m, int kq) {
  if (r >= m || t >= kq || r < t) return czero<R>();
  if (r == t) return mkc<R>(R(1), R(0));
  return Vp[(size_t)t * ld + r];
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
  if (gr >= m || gc >= m) return czero<R>();
  if (gr > gc) return A22[(size_t)gc * ld + gr];
  if (gr < gc) return conj(A22[(size_t)gr * ld + gc]);
  return mkc<R>(A22[(size_t)gc * ld + gr].re, R(0));
}

template <typename R>
__global__ void __launch_bounds__(256) he2hb_hemm(const EigItem *__restrict__ items, int p) {
  typedef cx<R> C;
  constexpr int TC = 32;
  constexpr int PER = 64 * TC / 256;   // tile elements loaded per thread
  __shared__ C tile[TC][65];        // tile[cc][rr] = A22(rb*64 + rr, cb*TC + cc)
  __shared__ C Vc[TC][HB];          // V rows of the column block
  const EigItem it = items[blockIdx.y];
  const int n = 2 * it.N, c0 = p * HB, m = n - c0 - HB;
  const int rb = blockIdx.x;
  if (m <= 0 || rb * 64 >= m) return;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  const C *__restrict__ A22 = (const C *)it.A + (size_t)(c0 + HB) * ld + (c0 + HB);
  const C *__restrict__ Vp = (const C *)it.A + (size_t)c0 * ld + (c0 + HB);
  const int tid = threadIdx.x, r = tid & 63, ks = tid >> 6;
  const int r0 = rb * 64;
  // Element e = tid + 256 u of a 64 x TC tile: below the row block it is read
  // down a stored column (rr fastest), right of it across (cc fastest, then
  // conjugate-transposed) so that both reads are coalesced.
  C nxt[PER], vnx[2];
  auto fetch = [&](int cb0) {
    const bool above = cb0 >= r0 + 64;   // entirely right of the diagonal block
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      int rr, cc;
      if (above) { cc = e % TC; rr = e / TC; } else { rr = e & 63; cc = e >> 6; }
      nxt[u] = hemm_elem<R>(A22, ld, m, r0 + rr, cb0 + cc);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + 256 * u;
      vnx[u] = panel_v<R>(Vp, ld, cb0 + e % TC, e / TC, m, kq);
    }
  };
  C acc[HB];
#pragma unroll
  for (int t = 0; t < HB; ++t) acc[t] = czero<R>();
  fetch(0);
  for (int cb0 = 0; cb0 < m; cb0 += TC) {
    const bool above = cb0 >= r0 + 64;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      int rr, cc;
      if (above) { cc = e % TC; rr = e / TC; } else { rr = e & 63; cc = e >> 6; }
      tile[cc][rr] = nxt[u];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + 256 * u;
      Vc[e % TC][e / TC] = vnx[u];
    }
    __syncthreads();
    if (cb0 + TC < m) fetch(cb0 + TC);   // in flight during the products below
#pragma unroll 2
    for (int cc = ks; cc < TC; cc += 4) {
      const C a = tile[cc][r];
#pragma unroll
      for (int t = 0; t < HB; ++t) acc[t] = cfma(a, Vc[cc][t], acc[t]);
    }
    __syncthreads();
  }
  // sum the 4 column phases (two halves of HB through the tile buffer)
  C *red = &tile[0][0];   // [4][64][HB/2]
  C *X0 = (C *)it.X0;
  __shared__ C X0s[64][HB + 1];
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int t = 0; t < HB / 2; ++t) red[(ks * 64 + r) * (HB / 2) + t] = acc[h * (HB / 2) + t];
    __syncthreads();
    for (int e = tid; e < 64 * (HB / 2); e += 256) {
      const int rr = e % 64, t = e / 64;
      C sm = czero<R>();
#pragma unroll
      for (int q = 0; q < 4; ++q) sm = sm + red[(q * 64 + rr) * (HB / 2) + t];
      X0s[rr][h * (HB / 2) + t] = sm;
      if (r0 + rr < m) X0[(size_t)(h * (HB / 2) + t) * ld + r0 + rr] = sm;
    }
    __syncthreads();
  }
  // Gram partial G[i][j] = sum_rr conj(V[rr][i]) X0[rr][j]; V rows of this
  // block staged through the tile buffer
  C *Vr = &tile[0][0];   // [64][HB]
  for (int e = tid; e < 64 * HB; e += 256) {
    const int i = e & 63, t = e >> 6;
    Vr[i * HB + t] = panel_v<R>(Vp, ld, r0 + i, t, m, kq);
  }
  __syncthreads();
  C *M0p = (C *)it.M0p + (size_t)rb * HB * HB;
  for (int e = tid; e < HB * HB; e += 256) {
    const int i = e % HB, jx = e / HB;
    C sm = czero<R>();
    for (int rr = 0; rr < 64; ++rr) sm = cfma_cj(Vr[rr * HB + i], X0s[rr][jx], sm);
    M0p[e] = sm;
  }
}

// ---------------------------------------------------------------------------
// Stage 1c.  W = X0 T - V Y / 2 with Y = T^H (V^H X0) T, for row block rb.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) he2hb_wform(const EigItem *__restrict__ items, int p) {
  typedef cx<R> C;
  __shared__ C G[HB][HB + 1], Tm[HB][HB + 1], Q1[HB][HB + 1], Y[HB][HB + 1];
  const EigItem it = items[blockIdx.y];
  const int n = 2 * it.N, c0 = p * HB, m = n - c0 - HB;
  const int rb = blockIdx.x;
  if (m <= 0 || rb * 64 >= m) return;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  const int tid = threadIdx.x;
  const int nrb = (m + 63) / 64;
  const C *M0p = (const C *)it.M0p;
  const C *T1 = (const C *)it.T1 + (size_t)p * HB * HB;
  for (int e = tid; e < HB * HB; e += 256) {
    const int i = e % HB, jx = e / HB;
    C s = czero<R>();
    for (int b = 0; b < nrb; ++b) s = s + M0p[(size_t)b * HB * HB + e];
    G[i][jx] = s;
    Tm[i][jx] = T1[e];
  }
  __syncthreads();
  for (int e = tid; e < HB * HB; e += 256) {
    const int i = e % HB, jx = e / HB;
    C s = czero<R>();
    for (int l = 0; l <= jx; ++l) s = cfma(G[i][l], Tm[l][jx], s);
    Q1[i][jx] = s;
  }
  __syncthreads();
  for (int e = tid; e < HB * HB; e += 256) {
    const int i = e % HB, jx = e / HB;
    C s = czero<R>();
    for (int l = 0; l <= i; ++l) s = cfma_cj(Tm[l][i], Q1[l][jx], s);
    Y[i][jx] = s;
  }
  __syncthreads();
  const C *X0 = (const C *)it.X0;
  const C *Vp = (const C *)it.A + (size_t)c0 * ld + (c0 + HB);
  C *Wm = (C *)it.Wm;
  const int rr = tid & 63, tq = tid >> 6;
  const int r = rb * 64 + rr;
  if (r >= m) return;
  C xr[HB], vr[HB];
#pragma unroll
  for (int t = 0; t < HB; ++t) {
    xr[t] = X0[(size_t)t * ld + r];
    vr[t] = panel_v<R>(Vp, ld, r, t, m, kq);
  }
#pragma unroll
  for (int tt = 0; tt < HB / 4; ++tt) {
    const int t = tq * (HB / 4) + tt;
    C s = czero<R>();
#pragma unroll
    for (int l = 0; l < HB; ++l) {
      if (l <= t) s = cfma(xr[l], Tm[l][t], s);
      s = s - R(0.5) * (vr[l] * Y[l][t]);
    }
    Wm[(size_t)t * ld + r] = s;
  }
}

// ---------------------------------------------------------------------------
// Stage 1d.  A22 <- A22 - W V^H - V W^H on the lower 64 x 64 tiles
// (upper entries of diagonal tiles are written too but never read).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) he2hb_her2k(const EigItem *__restrict__ items, int p) {
  typedef cx<R> C;
  __shared__ C Vr[HB][65], Wr[HB][65], Vc[HB][65], Wc[HB][65];
  const EigItem it = items[blockIdx.y];
  const int n = 2 * it.N, c0 = p * HB, m = n - c0 - HB;
  if (m <= 0) return;
  const int nt = (m + 63) / 64;
  const int t = blockIdx.x;
  if (t >= nt * (nt + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int kq = min(m, HB);
  const size_t ld = (size_t)n;
  C *__restrict__ A22 = (C *)it.A + (size_t)(c0 + HB) * ld + (c0 + HB);
  const C *__restrict__ Vp = (const C *)it.A + (size_t)c0 * ld + (c0 + HB);
  const C *__restrict__ Wm = (const C *)it.Wm;
  const int r0 = I * 64, cc0 = J * 64;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  for (int e = tid; e < 64 * HB; e += 256) {
    const int i = e & 63, k = e >> 6;
    const int gr = r0 + i, gc = cc0 + i;
    const bool kr = k < kq;
    Vr[k][i] = panel_v<R>(Vp, ld, gr, k, m, kq);
    Wr[k][i] = (gr < m && kr) ? Wm[(size_t)k * ld + gr] : czero<R>();
    Vc[k][i] = (gc < m && kr) ? conj(Wm[(size_t)k * ld + gc]) : czero<R>();
    Wc[k][i] = conj(panel_v<R>(Vp, ld, gc, k, m, kq));
  }
  // the output tile is fetched before the product so that its latency overlaps it
  C cur[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int gc = cc0 + ty + 16 * b;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int gr = r0 + tx + 16 * a;
      cur[a][b] = (gc < m && gr < m) ? A22[(size_t)gc * ld + gr] : czero<R>();
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < HB; ++k) {
    C a1[4], a2[4], b1[4], b2[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      a1[a] = -Vr[k][tx + 16 * a];
      a2[a] = -Wr[k][tx + 16 * a];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      b1[b] = Vc[k][ty + 16 * b];
      b2[b] = Wc[k][ty + 16 * b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cur[a][b] = cfma(a1[a], b1[b], cfma(a2[a], b2[b], cur[a][b]));
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int gc = cc0 + ty + 16 * b;
    if (gc >= m) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int gr = r0 + tx + 16 * a;
      if (gr >= m) continue;
      A22[(size_t)gc * ld + gr] = cur[a][b];
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
MVPB_DEV cx<R> shfl_xor_c(cx<R> v, int o) {
  return mkc<R>(__shfl_xor(v.re, o, 64), __shfl_xor(v.im, o, 64));
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
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
MVPB_DEV float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
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
constexpr int CH_WAVES = 16;
constexpr long long CH_SPIN_LIMIT = 1ll << 24;

template <typename R>
__global__ void __launch_bounds__(CH_WAVES * 64) hb2st(const EigItem *__restrict__ items) {
  typedef cx<R> C;
  __shared__ int prog[CH_WAVES];
  __shared__ int abort_s;
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N;
  const size_t ld = (size_t)n;
  const C *__restrict__ A = (const C *)it.A;
  C *__restrict__ WB = (C *)it.WB;
  C *__restrict__ V2 = (C *)it.V2;
  C *__restrict__ tau2 = (C *)it.tau2;
  const int tid = threadIdx.x;
  for (size_t e = tid; e < (size_t)n * HB_LDB; e += CH_WAVES * 64) {
    const int c = (int)(e / HB_LDB), d = (int)(e % HB_LDB), r = c + d;
    C v = czero<R>();
    if (d <= HB && r < n) {
      v = A[(size_t)c * ld + r];
      if (d == 0) v.im = R(0);
    }
    WB[e] = v;
  }
  if (tid < CH_WAVES) prog[tid] = -1;
  if (tid == 0) {
    abort_s = 0;
    *it.flag = 0;
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63, q = lane & 15, g = lane >> 4;
  bool aborted = false;
  for (int i = w; i < n - 1 && !aborted; i += CH_WAVES) {
    const int nsteps = (n - 1 - i + HB - 1) / HB;
    const int nprev = (n - i + HB - 1) / HB;   // blocks of sweep i-1
    const long long roff = refl_count(n - 1) - refl_count(n - 1 - i);
    C vprev = czero<R>(), tauprev = czero<R>();
    for (int k = 0; k < nsteps; ++k) {
      if (i > 0) {
        const int need = (i - 1) * 1024 + min(k + 3, nprev);
        long long spins = 0;
        while (__hip_atomic_load(&prog[(i - 1) % CH_WAVES], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
          if (__hip_atomic_load(&abort_s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            aborted = true;
            break;
          }
          if (++spins > CH_SPIN_LIMIT) {
            __hip_atomic_store(&abort_s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lane == 0) *it.flag = 1;
            aborted = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (aborted) break;
      }
      const int s = i + 1 + k * HB;
      const int L = min(HB, n - s);
      const int ps = s - HB;   // J_{k-1} = [s-HB, s-1] (k >= 1)
      // ---- every load of the task at once: the column / block being
      // annihilated and the diagonal block D = A[J_k, J_k]
      C y[4], dq[4];
      if (k == 0) {
        const C x = (q < L) ? WB[(size_t)i * HB_LDB + 1 + q] : czero<R>();
#pragma unroll
        for (int t = 0; t < 4; ++t) y[t] = x;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = 4 * g + t;
          y[t] = (q < L) ? WB[(size_t)(ps + c) * HB_LDB + HB + q - c] : czero<R>();
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = 4 * g + t;
        C v = czero<R>();
        if (q < L && c < L) {
          if (q >= c) v = WB[(size_t)(s + c) * HB_LDB + q - c];
          else v = conj(WB[(size_t)(s + q) * HB_LDB + c - q]);
        }
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
        yv = yv + shfl_xor_c(yv, 16);
        yv = yv + shfl_xor_c(yv, 32);
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
        if (g == 0 && q < L) WB[(size_t)i * HB_LDB + 1 + q] = betac;
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
            WB[(size_t)(ps + c) * HB_LDB + HB + q - c] = y[t];
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
        w0 = w0 + shfl_xor_c(w0, 16);
        w0 = w0 + shfl_xor_c(w0, 32);
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
              WB[(size_t)(s + c) * HB_LDB + q - c] = v;
            }
          }
        }
      }
      __threadfence_block();
      if (lane == 0)
        __hip_atomic_store(&prog[w], i * 1024 + k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      // the reflector for the back-transform (after the release: not waited for)
      if (g == 0) {
        C *dst = V2 + (size_t)(roff + k) * HB + q;
        __builtin_nontemporal_store(vq.re, &dst->re);
        __builtin_nontemporal_store(vq.im, &dst->im);
      }
      if (lane == 0) tau2[roff + k] = tau;
      vprev = vq;
      tauprev = tau;
    }
  }
  __syncthreads();
  if (abort_s) return;
  for (int r = tid; r < n; r += CH_WAVES * 64) {
    it.d[r] = (double)WB[(size_t)r * HB_LDB].re;
    if (r < n - 1) it.e[r] = (double)WB[(size_t)r * HB_LDB + 1].re;
  }
}

// ---------------------------------------------------------------------------
// Back-transform.  Z (n x nc columns of the tridiagonal eigenvectors) in LDS;
// apply the stage-2 reflectors sweep by sweep from the last, then the stage-1
// block reflectors panel by panel from the last.  Output Y (complex, n x nb,
// column-major) in the reduction precision.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(BT_THREADS) backtransform_2s(const EigItem *__restrict__ items, int nc) {
  typedef cx<R> C;
  extern __shared__ __align__(16) unsigned char shraw[];
  C *Z = (C *)shraw;   // Z[r * nc + c]
  __shared__ C S[HB][8], S2[HB][8], Tm[HB][HB + 1];
  const EigItem it = items[blockIdx.y];
  const int n = 2 * it.N, nb = it.nb;
  const int cbase = blockIdx.x * nc;
  if (cbase >= nb) return;
  const int ncl = min(nc, nb - cbase);
  const int tid = threadIdx.x;
  const size_t ld = (size_t)n;
  for (int e = tid; e < n * nc; e += BT_THREADS) {
    const int r = e / nc, c = e % nc;
    Z[e] = (c < ncl) ? mkc<R>((R)it.X[(size_t)r * nb + cbase + c], R(0)) : czero<R>();
  }
  __syncthreads();
  // ---- stage 2: sweeps i = n-2 .. 0; the blocks of one sweep are disjoint.
  // Thread e owns the (block, column) pair (e / ncl, e % ncl) of every sweep;
  // the reflector of the next sweep is loaded while this one is applied.
  const C *V2 = (const C *)it.V2;
  const C *tau2 = (const C *)it.tau2;
  const long long rtot = refl_count(n - 1);
  auto fetch = [&](int i, C (&vv)[HB], C &tau) {
    const int nsteps = (n - 1 - i + HB - 1) / HB;
    const int k = tid / ncl;
    if (i < 0 || k >= nsteps) return;
    const long long ri = rtot - refl_count(n - 1 - i) + k;
    const C *v = V2 + (size_t)ri * HB;
    const int L = min(HB, n - (i + 1 + k * HB));
#pragma unroll
    for (int j = 0; j < HB; ++j) vv[j] = (j < L) ? v[j] : czero<R>();
    tau = tau2[ri];
  };
  C vcur[HB], vnxt[HB], tcur = czero<R>(), tnxt = czero<R>();
#pragma unroll
  for (int j = 0; j < HB; ++j) vcur[j] = vnxt[j] = czero<R>();
  fetch(n - 2, vcur, tcur);
  for (int i = n - 2; i >= 0; --i) {
    fetch(i - 1, vnxt, tnxt);
    const int nsteps = (n - 1 - i + HB - 1) / HB;
    const int k = tid / ncl, c = tid % ncl;
    if (k < nsteps) {
      const int s = i + 1 + k * HB;
      const int L = min(HB, n - s);
      C *zc = Z + (size_t)s * nc + c;
      C d0 = czero<R>(), d1 = czero<R>();
#pragma unroll
      for (int j = 0; j < HB; j += 2) {
        if (j < L) d0 = cfma_cj(vcur[j], zc[(size_t)j * nc], d0);
        if (j + 1 < L) d1 = cfma_cj(vcur[j + 1], zc[(size_t)(j + 1) * nc], d1);
      }
      const C td = tcur * (d0 + d1);
#pragma unroll
      for (int j = 0; j < HB; ++j)
        if (j < L) zc[(size_t)j * nc] = zc[(size_t)j * nc] - vcur[j] * td;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < HB; ++j) vcur[j] = vnxt[j];
    tcur = tnxt;
  }
  // ---- stage 1: panels last to first; rows c0+HB .. n-1
  const int npan = n > HB ? (n - 1) / HB : 0;   // panels with m = n - p HB - HB > 0
  const C *A = (const C *)it.A;
  const int rg = tid & 15, tt = (tid >> 4) & (HB - 1);   // (row phase, reflector column) for V^H Z
  for (int p = npan - 1; p >= 0; --p) {
    const int c0 = p * HB, m = n - c0 - HB;
    const int kq = min(m, HB);
    const C *Vp = A + (size_t)c0 * ld + (c0 + HB);
    const C *T1 = (const C *)it.T1 + (size_t)p * HB * HB;
    for (int e = tid; e < HB * HB; e += BT_THREADS) Tm[e % HB][e / HB] = T1[e];
    // S = V^H Z[rows]: thread (rg, tt) sums rows rg, rg+16, ...
    C acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = czero<R>();
    if (tt < kq && tid < 16 * HB) {
      for (int r = tt + rg; r < m; r += 16) {   // V(r, tt) = 0 for r < tt
        const C v = (r == tt) ? mkc<R>(R(1), R(0)) : Vp[(size_t)tt * ld + r];
        const C *zr = Z + (size_t)(c0 + HB + r) * nc;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < ncl) acc[c] = cfma_cj(v, zr[c], acc[c]);
      }
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
      for (int c = 0; c < 8; ++c) acc[c] = acc[c] + shfl_xor_c(acc[c], o);
    }
    if (rg == 0 && tid < 16 * HB) {
#pragma unroll
      for (int c = 0; c < 8; ++c) S[tt][c] = acc[c];
    }
    __syncthreads();
    // S2 = T S
    for (int e = tid; e < HB * 8; e += BT_THREADS) {
      const int a = e / 8, c = e % 8;
      C s2 = czero<R>();
      if (a < kq)
        for (int l = a; l < kq; ++l) s2 = cfma(Tm[a][l], S[l][c], s2);
      S2[a][c] = s2;
    }
    __syncthreads();
    // Z[rows] -= V S2
    for (int e = tid; e < m * ncl; e += BT_THREADS) {
      const int r = e / ncl, c = e % ncl;
      C s2 = czero<R>();
      const int lmax = min(kq - 1, r);
      for (int l = 0; l <= lmax; ++l) {
        const C v = (r == l) ? mkc<R>(R(1), R(0)) : Vp[(size_t)l * ld + r];
        s2 = cfma(v, S2[l][c], s2);
      }
      C *z = Z + (size_t)(c0 + HB + r) * nc + c;
      *z = *z - s2;
    }
    __syncthreads();
  }
  C *Y = (C *)it.Yb;
  for (int e = tid; e < n * ncl; e += BT_THREADS) {
    const int r = e % n, c = e / n;
    const C z = Z[(size_t)r * nc + c];
    Y[(size_t)(cbase + c) * ld + r] = z;
    if (sizeof(R) != sizeof(double)) it.Y[(size_t)(cbase + c) * ld + r] = ccast<double>(z);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// The panel kernel's register blocking (RPT rows per thread) follows each
// item's own panel height, so an item's arithmetic does not depend on the
// other items of the launch: one launch per height class present, and the
// items of the other classes return at once.
template <typename R, int RPT>
static void launch_panel_class(const EigItem *items, int n_items, int p, int m_lo, int m_hi, hipStream_t st) {
  const int lo = (RPT / 2) * PQ_THREADS, hi = RPT * PQ_THREADS;   // class: lo < m <= hi
  if (m_hi <= lo || m_lo > hi) return;
  hipLaunchKernelGGL((he2hb_panel<R, RPT>), dim3(n_items), dim3(PQ_THREADS), 0, st, items, p);
}

template <typename R>
static hipError_t launch_reduce_t(const EigItem *items, int n_items, int n_min, int n_max, hipStream_t st) {
  for (int p = 0;; ++p) {
    const int c0 = p * HB, m = n_max - c0 - HB;
    if (m <= 0) break;
    const int m_lo = std::max(1, n_min - c0 - HB);
    {
      ProfScope ps(K_PANEL, st);
      launch_panel_class<R, 1>(items, n_items, p, m_lo, m, st);
      launch_panel_class<R, 2>(items, n_items, p, m_lo, m, st);
      launch_panel_class<R, 4>(items, n_items, p, m_lo, m, st);
      launch_panel_class<R, 8>(items, n_items, p, m_lo, m, st);
    }
    const int nrb = (m + 63) / 64;
    {
      ProfScope ps(K_HEMM, st);
      hipLaunchKernelGGL((he2hb_hemm<R>), dim3(nrb, n_items), dim3(256), 0, st, items, p);
    }
    {
      ProfScope ps(K_WFORM, st);
      hipLaunchKernelGGL((he2hb_wform<R>), dim3(nrb, n_items), dim3(256), 0, st, items, p);
    }
    {
      ProfScope ps(K_HER2K, st);
      hipLaunchKernelGGL((he2hb_her2k<R>), dim3(nrb * (nrb + 1) / 2, n_items), dim3(256), 0, st, items, p);
    }
  }
  {
    ProfScope ps(K_HB2ST, st);
    hipLaunchKernelGGL((hb2st<R>), dim3(n_items), dim3(CH_WAVES * 64), 0, st, items);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const EigItem *items, int n_items, int n_min, int n_max, bool fp32, hipStream_t st) {
  return fp32 ? launch_reduce_t<float>(items, n_items, n_min, n_max, st)
              : launch_reduce_t<double>(items, n_items, n_min, n_max, st);
}

// Eigenvector columns per back-transform workgroup: bounded by the LDS
// budget and by one (block, column) pair of a stage-2 sweep per thread.
int backtransform_cols(int n_max, bool fp32) {
  const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
  const size_t cap = (size_t)BT_LDS_BYTES / (es * (size_t)n_max);
  const size_t blocks = (size_t)std::max(1, (n_max - 1 + HB - 1) / HB);
  const size_t cap2 = (size_t)BT_THREADS / blocks;
  return (int)std::min<size_t>(8, std::max<size_t>(1, std::min(cap, cap2)));
}

hipError_t launch_backtransform(const EigItem *items, int n_items, int n_max, int nb, bool fp32, hipStream_t st) {
  ProfScope ps(K_BACKTRANSFORM, st);
  const int nc = backtransform_cols(n_max, fp32);
  const int groups = (nb + nc - 1) / nc;
  const size_t es = fp32 ? sizeof(cf) : sizeof(cd);
  const size_t sh = es * (size_t)n_max * nc;
  if (fp32)
    hipLaunchKernelGGL((backtransform_2s<float>), dim3(groups, n_items), dim3(BT_THREADS), sh, st, items, nc);
  else
    hipLaunchKernelGGL((backtransform_2s<double>), dim3(groups, n_items), dim3(BT_THREADS), sh, st, items, nc);
  return hipGetLastError();
}

hipError_t init_band_attributes() {
  hipError_t e = hipFuncSetAttribute((const void *)backtransform_2s<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, BT_LDS_BYTES);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)backtransform_2s<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             BT_LDS_BYTES);
}

}  // namespace mvpb
