// Batched Hermitian eigensolve for the lowest bands of C(k) (2N x 2N).
//
//  1. Blocked Householder reduction to real symmetric tridiagonal form
//     (C = Q T Q^H).  Per panel of PANEL columns: one workgroup per item
//     builds the reflectors and the panel matrix W (the matrix-vector
//     product with the trailing matrix is the bandwidth-bound part), then a
//     tiled kernel spread over the whole GPU applies the rank-2*PANEL update
//     A <- A - V W^H - W V^H to every item's trailing matrix.
//  2. Lowest nb eigenvalues of T by multisection on Sturm counts; their
//     eigenvectors by inverse iteration with a pivoted tridiagonal LU,
//     re-orthonormalised as a block after each sweep.
//  3. Back-transform Y = Q X with the stored reflectors.
//  4. FP64 Rayleigh-Ritz on span(Y) with the kept copy of C(k):
//     eigenpairs of Y^H C Y, omega = sqrt(max(lambda, 0)).
#include <float.h>

#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

constexpr int EIG_THREADS = 1024;
constexpr int EIG_WAVES = EIG_THREADS / 64;
// Panel kernel: columns of the trailing matrix consumed per load batch.
constexpr int PANEL_THREADS = 1024;
constexpr int PANEL_WAVES = PANEL_THREADS / 64;
static_assert(PANEL_WAVES == PANEL_SLOTS, "one partial-sum slot per panel wave");
constexpr int COLS = 8;

// Sum 8 complex values over the 64 lanes of a wavefront, one value per
// column: after the butterfly, lanes with (lane >> 3) & 7 == k hold the sum
// of column k.  Contents of v are destroyed.
template <typename R>
MVPB_DEV cx<R> reduce8_columns(cx<R> (&v)[8], int lane) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool hi = lane & 32;
    cx<R> snd = hi ? v[k] : v[k + 4];
    const cx<R> keep = hi ? v[k + 4] : v[k];
    snd.re = __shfl_xor(snd.re, 32, 64);
    snd.im = __shfl_xor(snd.im, 32, 64);
    v[k] = keep + snd;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const bool hi = lane & 16;
    cx<R> snd = hi ? v[k] : v[k + 2];
    const cx<R> keep = hi ? v[k + 2] : v[k];
    snd.re = __shfl_xor(snd.re, 16, 64);
    snd.im = __shfl_xor(snd.im, 16, 64);
    v[k] = keep + snd;
  }
  {
    const bool hi = lane & 8;
    cx<R> snd = hi ? v[0] : v[1];
    const cx<R> keep = hi ? v[1] : v[0];
    snd.re = __shfl_xor(snd.re, 8, 64);
    snd.im = __shfl_xor(snd.im, 8, 64);
    v[0] = keep + snd;
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) {
    v[0].re += __shfl_xor(v[0].re, o, 64);
    v[0].im += __shfl_xor(v[0].im, o, 64);
  }
  return v[0];
}

// ---------------------------------------------------------------------------
// 1a. Panel kernel: columns p .. p+nbp-1 of every item.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(PANEL_THREADS) hetrd_panel(const EigItem *__restrict__ items, int p, int nmax) {
  typedef cx<R> C;
  typedef const __attribute__((address_space(1))) C gC;
  extern __shared__ __align__(16) unsigned char shraw[];
  C *v = (C *)shraw;                            // nmax: current reflector (rows j+1..n-1)
  R *yr = (R *)(v + nmax);              // nmax: real parts of the new W column
  R *yi = yr + nmax;                    // nmax: imaginary parts
  __shared__ double red[2 * PANEL_WAVES];
  __shared__ C t1[PANEL], t2[PANEL], wj[PANEL], vj[PANEL];
  __shared__ C colsum[PANEL_WAVES * 64];
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N;
  if (p >= n - 1) return;
  const int nbp = min(PANEL, n - 1 - p);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  C *__restrict__ A = (C *)it.A;
  C *__restrict__ W = (C *)it.W;
  const size_t ld = (size_t)n;

  for (int i = 0; i < nbp; ++i) {
    const int j = p + i;
    // --- step 1: bring column j up to date with the panel's earlier reflectors
    if (tid < i) {
      wj[tid] = conj(W[(size_t)tid * ld + j]);
      vj[tid] = conj(A[(size_t)(p + tid) * ld + j]);
    }
    __syncthreads();
    for (int r = j + tid; r < n; r += PANEL_THREADS) {
      C acc = A[(size_t)j * ld + r];
      for (int k0 = 0; k0 < i; k0 += 8) {
        C av[8], wv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const bool ok = k0 + k < i;
          av[k] = ok ? A[(size_t)(p + k0 + k) * ld + r] : czero<R>();
          wv[k] = ok ? W[(size_t)(k0 + k) * ld + r] : czero<R>();
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (k0 + k < i) {
            acc = acc - av[k] * wj[k0 + k];
            acc = acc - wv[k] * vj[k0 + k];
          }
        }
      }
      if (r == j) acc.im = R(0);
      A[(size_t)j * ld + r] = acc;
    }
    __syncthreads();
    // --- step 2: reflector annihilating A[j+2:n, j]
    double xn2 = 0.0;
    for (int r = j + 2 + tid; r < n; r += PANEL_THREADS) xn2 += (double)abs2(A[(size_t)j * ld + r]);
    xn2 = block_sum(xn2, red);
    const C alpha = A[(size_t)j * ld + j + 1];
    C tau = czero<R>(), scale = czero<R>();
    double beta = (double)alpha.re;
    if (!(xn2 == 0.0 && alpha.im == R(0))) {
      const double ar = alpha.re, ai = alpha.im;
      const double nrm = sqrt(ar * ar + ai * ai + xn2);
      beta = ar >= 0.0 ? -nrm : nrm;
      tau = mkc<R>((R)((beta - ar) / beta), (R)(-ai / beta));
      scale = ccast<R>(cdiv(mk(1.0, 0.0), mk(ar - beta, ai)));
    }
    const int m = n - j - 1;
    for (int r = j + 1 + tid; r < n; r += PANEL_THREADS) {
      C x;
      if (r == j + 1) {
        x = mkc<R>(R(1), R(0));
      } else {
        x = A[(size_t)j * ld + r] * scale;
      }
      A[(size_t)j * ld + r] = x;
      v[r - j - 1] = x;
    }
    if (tid == 0) {
      it.d[j] = (double)A[(size_t)j * ld + j].re;
      it.e[j] = (double)(R)beta;
      ((C *)it.tau)[j] = tau;
    }
    __syncthreads();
    // --- step 3: y = A22 v with A22 = A[j+1:, j+1:] (pre-panel values).
    // Hermitian product from the lower triangle only: 64 x 64 tiles (s >= cb)
    // spread over the waves; a lane owns one row, COLS columns are loaded at
    // a time, the row sums stay in the lane and the column sums (conjugate
    // side) are folded across lanes by a butterfly.  Each wave accumulates
    // into its own slot; the slots are summed in a fixed order, so the result
    // is bitwise reproducible.
    const C *A22 = A + (size_t)(j + 1) * ld + (j + 1);
    // this wave's partial sums: row side and conjugate (column) side kept
    // apart, so that every entry is only ever touched by one lane
    C *ywr = (C *)it.Yw + (size_t)(2 * w) * ld;
    C *ywc = ywr + ld;
    for (int r = lane; r < m; r += 64) ywr[r] = czero<R>();
    // column c of a chunk is written by lane 8 (c % 8); clear it with that lane
    if ((lane & 7) == 0)
      for (int c = lane >> 3; c < m; c += 8) ywc[c] = czero<R>();
    {
      // tiles in column-major order over the lower triangle, a contiguous
      // range per wave, so a wave stays on one column block for long runs and
      // keeps that block's conjugate-side sums in registers
      const int S = (m + 63) / 64;
      const int ntile = S * (S + 1) / 2;
      const int t0 = (int)((long)ntile * w / PANEL_WAVES), t1 = (int)((long)ntile * (w + 1) / PANEL_WAVES);
      int cb = 0, s = 0;
      {
        int t = t0;
        while (t >= S - cb) { t -= S - cb; ++cb; }
        s = cb + t;
      }
      // conjugate-side sums of the current column block: 64 per wave in LDS,
      // slot q*8 + k only ever touched by lane 8k
      C *colacc = colsum + w * 64;
      if ((lane & 7) == 0)
        for (int q = 0; q < 8; ++q) colacc[q * 8 + (lane >> 3)] = czero<R>();
      for (int t = t0; t < t1; ++t) {
        const int r = s * 64 + lane;
        const bool rv = r < m;
        const int rc = rv ? r : m - 1;                 // clamped row: loads stay inside the matrix
        const C vr = rv ? v[r] : czero<R>();
        const bool diag = (s == cb);                    // uniform per tile
        C accr = czero<R>();
        const int cend = min(cb * 64 + 64, m);
        const gC *colp = (const gC *)(A22 + (size_t)(cb * 64) * ld + rc);
#pragma unroll 1
        for (int q = 0; q < 8; ++q) {
          const int c0 = cb * 64 + q * COLS;
          if (c0 >= cend) break;
          const int kmax = min(COLS, cend - c0);        // uniform
          C a[COLS];
#pragma unroll
          for (int k = 0; k < COLS; ++k) {
            if (k < kmax) {
              const gC *pq = colp + (size_t)(q * COLS + k) * ld;
              a[k] = mkc<R>(pq->re, pq->im);
            } else {
              a[k] = czero<R>();
            }
          }
          if (!diag) {
#pragma unroll
            for (int k = 0; k < COLS; ++k) {
              const C vc = (k < kmax) ? v[c0 + k] : czero<R>();
              accr = cfma(a[k], vc, accr);
              a[k] = cfma_cj(a[k], vr, czero<R>());   // conjugate side
            }
          } else {
            // diagonal tile: lower triangle only, the diagonal counted once
#pragma unroll
            for (int k = 0; k < COLS; ++k) {
              const int c = c0 + k;
              const R wt = (k < kmax && r >= c) ? R(1) : R(0);
              const R wc = (k < kmax && r > c) ? R(1) : R(0);
              const C vc = (k < kmax) ? v[c] : czero<R>();
              accr = cfma(wt * a[k], vc, accr);
              a[k] = wc * cfma_cj(a[k], vr, czero<R>());
            }
          }
          const C cs = reduce8_columns<R>(a, lane);
          if ((lane & 7) == 0) colacc[q * 8 + (lane >> 3)] = colacc[q * 8 + (lane >> 3)] + cs;
        }
        if (rv) ywr[r] = ywr[r] + accr;
        // next tile; flush the column sums when the column block changes
        ++s;
        if (s >= S || t + 1 == t1) {
          if ((lane & 7) == 0) {
            for (int q = 0; q < 8; ++q) {
              const int c = cb * 64 + q * COLS + (lane >> 3);
              if (c < m) ywc[c] = ywc[c] + colacc[q * 8 + (lane >> 3)];
              colacc[q * 8 + (lane >> 3)] = czero<R>();
            }
          }
          if (s >= S) {
            ++cb;
            s = cb;
          }
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < m; r += PANEL_THREADS) {
      C acc = czero<R>();
#pragma unroll
      for (int q = 0; q < 2 * PANEL_WAVES; ++q) acc = acc + ((const C *)it.Yw)[(size_t)q * ld + r];
      yr[r] = acc.re;
      yi[r] = acc.im;
    }
    __syncthreads();
    // corrections with the panel's earlier columns (V = A[:, p:p+i], W[:, 0:i])
    if (i > 0) {
      for (int k = w; k < 2 * i; k += PANEL_WAVES) {
        const bool isW = k < i;
        const int kk = isW ? k : k - i;
        const C *col = isW ? (W + (size_t)kk * ld) : (A + (size_t)(p + kk) * ld);
        C acc = czero<R>();
#pragma unroll 8
        for (int r = j + 1 + lane; r < n; r += 64) acc = cfma_cj(col[r], v[r - j - 1], acc);
        acc.re = wave_sum(acc.re);
        acc.im = wave_sum(acc.im);
        if (lane == 0) {
          if (isW) t1[kk] = acc; else t2[kk] = acc;
        }
      }
      __syncthreads();
      for (int r = j + 1 + tid; r < n; r += PANEL_THREADS) {
        C acc = mkc<R>(yr[r - j - 1], yi[r - j - 1]);
        for (int k0 = 0; k0 < i; k0 += 8) {
          C av[8], wv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const bool ok = k0 + k < i;
            av[k] = ok ? A[(size_t)(p + k0 + k) * ld + r] : czero<R>();
            wv[k] = ok ? W[(size_t)(k0 + k) * ld + r] : czero<R>();
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (k0 + k < i) {
              acc = acc - av[k] * t1[k0 + k];
              acc = acc - wv[k] * t2[k0 + k];
            }
          }
        }
        yr[r - j - 1] = acc.re;
        yi[r - j - 1] = acc.im;
      }
      __syncthreads();
    }
    // y = tau y ; y += (-1/2 tau (y^H v)) v
    C dot = czero<R>();
    for (int r = tid; r < m; r += PANEL_THREADS) {
      const C yy = tau * mkc<R>(yr[r], yi[r]);
      yr[r] = yy.re;
      yi[r] = yy.im;
      dot = cfma_cj(yy, v[r], dot);
    }
    dot = block_sum_c(dot, red);
    const C al2 = mkc<R>(R(-0.5), R(0)) * tau * dot;
    for (int r = tid; r < m; r += PANEL_THREADS) {
      const C yy = cfma(al2, v[r], mkc<R>(yr[r], yi[r]));
      W[(size_t)i * ld + j + 1 + r] = yy;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 1b. Trailing update A[q0:, q0:] -= V W^H + W V^H, q0 = p + nbp, on the
//     lower triangle (upper entries of diagonal tiles are updated too but
//     never read).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) hetrd_update(const EigItem *__restrict__ items, int p) {
  typedef cx<R> C;
  constexpr int BK = 8;
  __shared__ C Vr[BK][65], Wr[BK][65], Vc[BK][65], Wc[BK][65];
  const EigItem it = items[blockIdx.z];
  const int n = 2 * it.N;
  if (p >= n - 1) return;
  const int nbp = min(PANEL, n - 1 - p);
  const int q0 = p + nbp, m = n - q0;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  // only the lower triangle (tiles with row block >= column block) is kept
  if (r0 >= m || c0 >= m || blockIdx.x < blockIdx.y) return;
  C *__restrict__ A = (C *)it.A;
  const C *__restrict__ W = (const C *)it.W;
  const size_t ld = (size_t)n;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  C acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = czero<R>();
  for (int k0 = 0; k0 < nbp; k0 += BK) {
    for (int e = tid; e < 64 * BK; e += 256) {
      const int i = e & 63, k = e >> 6;
      const int gk = k0 + k;
      const int gr = q0 + r0 + i, gc = q0 + c0 + i;
      C vr = czero<R>(), wr = vr, vc = vr, wc = vr;
      if (gk < nbp) {
        if (gr < n) {
          vr = A[(size_t)(p + gk) * ld + gr];
          wr = W[(size_t)gk * ld + gr];
        }
        if (gc < n) {
          vc = conj(W[(size_t)gk * ld + gc]);
          wc = conj(A[(size_t)(p + gk) * ld + gc]);
        }
      }
      Vr[k][i] = vr;
      Wr[k][i] = wr;
      Vc[k][i] = vc;
      Wc[k][i] = wc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      C a1[4], a2[4], b1[4], b2[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        a1[a] = Vr[k][tx + 16 * a];
        a2[a] = Wr[k][tx + 16 * a];
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        b1[b] = Vc[k][ty + 16 * b];
        b2[b] = Wc[k][ty + 16 * b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = cfma(a2[a], b2[b], cfma(a1[a], b1[b], acc[a][b]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int gc = q0 + c0 + ty + 16 * b;
    if (gc >= n) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int gr = q0 + r0 + tx + 16 * a;
      if (gr >= n) continue;
      C *dst = A + (size_t)gc * ld + gr;
      const C nv = *dst - acc[a][b];
      *dst = nv;
      // the last diagonal entry has no reflector; the last update fixes it
      if (gr == n - 1 && gc == n - 1) it.d[n - 1] = (double)nv.re;
    }
  }
}

template <typename R>
static hipError_t launch_hetrd_t(const EigItem *items, int n_items, int n_max, hipStream_t st) {
  const size_t sh = sizeof(cx<R>) * 2 * (size_t)n_max;
  for (int p = 0; p < n_max - 1; p += PANEL) {
    {
      ProfScope ps(K_HETRD_PANEL, st);
      hipLaunchKernelGGL(hetrd_panel<R>, dim3(n_items), dim3(PANEL_THREADS), sh, st, items, p, n_max);
    }
    const int nbp = min(PANEL, n_max - 1 - p);
    const int m = n_max - p - nbp;
    if (m > 0) {
      const int t = (m + 63) / 64;
      ProfScope ps(K_HETRD_UPDATE, st);
      hipLaunchKernelGGL(hetrd_update<R>, dim3(t, t, n_items), dim3(256), 0, st, items, p);
    }
  }
  return hipGetLastError();
}

hipError_t launch_hetrd(const EigItem *items, int n_items, int n_max, bool fp32, hipStream_t st) {
  return fp32 ? launch_hetrd_t<float>(items, n_items, n_max, st) : launch_hetrd_t<double>(items, n_items, n_max, st);
}

// ---------------------------------------------------------------------------
// 2. Tridiagonal eigenproblem: multisection for the lowest nb eigenvalues,
//    inverse iteration for the eigenvectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sturm_count(const double *dd, const double *ee2, int n, double x, double pivmin) {
  // number of eigenvalues of T strictly below x (LDL^T pivots)
  int cnt = 0;
  double q = dd[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int k = 1; k < n; ++k) {
    q = dd[k] - x - ee2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

__device__ __forceinline__ double hash_uniform(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h & 0xFFFFFF) / (double)0x1000000 * 2.0 - 1.0;
}

// Orthonormalise the nb columns of the real row-major block X[r*nb + b]
// (classical Gram-Schmidt, two passes).  Whole-block cooperative.
__device__ void orthonormalize_real(double *X, int n, int nb, double *h, double *red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int b = 0; b < nb; ++b) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = w; c < b; c += EIG_WAVES) {
        double acc = 0.0;
        for (int r = lane; r < n; r += 64) acc = fma(X[(size_t)r * nb + c], X[(size_t)r * nb + b], acc);
        acc = wave_sum(acc);
        if (lane == 0) h[c] = acc;
      }
      __syncthreads();
      for (int r = tid; r < n; r += EIG_THREADS) {
        double acc = X[(size_t)r * nb + b];
        for (int c = 0; c < b; ++c) acc = fma(-h[c], X[(size_t)r * nb + c], acc);
        X[(size_t)r * nb + b] = acc;
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int r = tid; r < n; r += EIG_THREADS) s = fma(X[(size_t)r * nb + b], X[(size_t)r * nb + b], s);
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int r = tid; r < n; r += EIG_THREADS) X[(size_t)r * nb + b] *= inv;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(EIG_THREADS) tridiag_eig(const EigItem *__restrict__ items) {
  extern __shared__ double shd[];
  double *dd = shd;            // MAX_N
  double *ee2 = dd + MAX_N;    // MAX_N: e^2
  double *ee = ee2 + MAX_N;    // MAX_N: e
  __shared__ double lo[64], hi[64], xs[EIG_THREADS];
  __shared__ int cnts[EIG_THREADS];
  __shared__ double red[2 * EIG_WAVES];
  __shared__ double h[64];
  __shared__ int done_s;
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N, nb = it.nb;
  const int tid = threadIdx.x;
  // stage d, e^2; Gershgorin bounds
  double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
  for (int r = tid; r < n; r += EIG_THREADS) {
    const double dr = it.d[r];
    const double er = (r < n - 1) ? it.e[r] : 0.0;
    const double el = (r > 0) ? it.e[r - 1] : 0.0;
    dd[r] = dr;
    if (r < n - 1) {
      ee2[r] = er * er;
      ee[r] = er;
    }
    const double rad = fabs(er) + fabs(el);
    gl = fmin(gl, dr - rad);
    gu = fmax(gu, dr + rad);
    emax2 = fmax(emax2, er * er);
  }
  // block min / max through the sum helper on transformed values
  {
    const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      gl = fmin(gl, __shfl_xor(gl, o, 64));
      gu = fmax(gu, __shfl_xor(gu, o, 64));
      emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
    }
    __shared__ double mm[3 * EIG_WAVES];
    if (lane == 0) { mm[3 * wid] = gl; mm[3 * wid + 1] = gu; mm[3 * wid + 2] = emax2; }
    __syncthreads();
    gl = DBL_MAX; gu = -DBL_MAX; emax2 = 0.0;
    for (int q = 0; q < EIG_WAVES; ++q) {
      gl = fmin(gl, mm[3 * q]);
      gu = fmax(gu, mm[3 * q + 1]);
      emax2 = fmax(emax2, mm[3 * q + 2]);
    }
    __syncthreads();
  }
  const double bnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  gl -= 2.0 * DBL_EPSILON * bnorm * n + 2.0 * pivmin;
  gu += 2.0 * DBL_EPSILON * bnorm * n + 2.0 * pivmin;
  if (tid < nb) { lo[tid] = gl; hi[tid] = gu; }
  __syncthreads();
  // multisection: G probes per wanted eigenvalue
  const int G = EIG_THREADS / nb;
  const int b = tid / G, g = tid % G;
  for (int round = 0; round < 24; ++round) {
    if (b < nb) {
      const double l = lo[b], hh = hi[b];
      const double x = l + (hh - l) * (double)(g + 1) / (double)(G + 1);
      xs[tid] = x;
      cnts[tid] = sturm_count(dd, ee2, n, x, pivmin);
    }
    __syncthreads();
    if (tid < nb) {
      const int base = tid * G;
      double nl = lo[tid], nh = hi[tid];
      int gg = 0;
      while (gg < G && cnts[base + gg] <= tid) ++gg;   // first probe with more than tid eigenvalues below
      if (gg < G) nh = xs[base + gg];
      if (gg > 0) nl = xs[base + gg - 1];
      lo[tid] = nl;
      hi[tid] = nh;
    }
    if (tid == 0) done_s = 1;
    __syncthreads();
    if (tid < nb) {
      const double tol = 2.0 * DBL_EPSILON * fmax(fabs(lo[tid]), fabs(hi[tid])) + 4.0 * pivmin;
      if (hi[tid] - lo[tid] > tol) atomicAnd(&done_s, 0);
    }
    __syncthreads();
    if (done_s) break;
    __syncthreads();
  }
  if (tid < nb) it.lam_t[tid] = 0.5 * (lo[tid] + hi[tid]);
  __syncthreads();
  // inverse iteration, one thread per eigenvalue; scratch lu[(a*n + r)*nb + b]
  double *lu = it.lu;
  double *X = it.X;
  // pivot used in place of an exact zero (the all-zero operator at Gamma with one plane wave)
  const double pert = fmax(DBL_EPSILON * bnorm, 1e-280);
  if (tid < nb) {
    const int bb = tid;
    const double lam = 0.5 * (lo[bb] + hi[bb]);
#define DL(r) lu[((size_t)0 * n + (r)) * nb + bb]
#define DG(r) lu[((size_t)1 * n + (r)) * nb + bb]
#define DU(r) lu[((size_t)2 * n + (r)) * nb + bb]
#define DU2(r) lu[((size_t)3 * n + (r)) * nb + bb]
#define PV(r) lu[((size_t)4 * n + (r)) * nb + bb]
    // LU with partial pivoting of T - lam I; the running row lives in
    // registers and the inputs come from LDS, so only stores go to memory
    double dr = dd[0] - lam, ur = (n > 1) ? ee[0] : 0.0;
    for (int r = 0; r < n - 1; ++r) {
      const double lr = ee[r];
      const double dn = dd[r + 1] - lam;
      const double un = (r < n - 2) ? ee[r + 1] : 0.0;
      if (fabs(dr) >= fabs(lr)) {
        const double piv = (dr == 0.0) ? pert : dr;
        const double f = lr / piv;
        DG(r) = piv; DU(r) = ur; DU2(r) = 0.0; DL(r) = f; PV(r) = 0.0;
        dr = dn - f * ur;
        ur = un;
      } else {
        const double f = dr / lr;
        DG(r) = lr; DU(r) = dn; DU2(r) = un; DL(r) = f; PV(r) = 1.0;
        dr = ur - f * dn;
        ur = -f * un;
      }
    }
    DG(n - 1) = (dr == 0.0) ? pert : dr;
    for (int r = 0; r < n; ++r) X[(size_t)r * nb + bb] = hash_uniform(r + 1, bb + 7);
  }
  for (int iter = 0; iter < 3; ++iter) {
    if (tid < nb) {
      const int bb = tid;
      // forward: apply P and L^-1; the running entry stays in a register
      double cur = X[bb];
      for (int r = 0; r < n - 1; ++r) {
        const double nxt = X[(size_t)(r + 1) * nb + bb];
        const bool sw = PV(r) != 0.0;
        const double br = sw ? nxt : cur;
        const double br1 = sw ? cur : nxt;
        X[(size_t)r * nb + bb] = br;
        cur = br1 - DL(r) * br;
      }
      X[(size_t)(n - 1) * nb + bb] = cur;
      // back substitution with U (diagonal, super and second super diagonal)
      double x1 = 0.0, x2 = 0.0, xmax = 0.0, sc = 1.0;
      for (int r = n - 1; r >= 0; --r) {
        double s = sc * X[(size_t)r * nb + bb];
        if (r + 1 < n) s -= DU(r) * x1;
        if (r + 2 < n) s -= DU2(r) * x2;
        double xv = s / DG(r);
        if (!isfinite(xv)) xv = 0.0;
        if (fabs(xv) > 1e150) {
          // keep the iterate finite: rescale what is solved and what is left
          const double f = 1e-150;
          for (int q = r + 1; q < n; ++q) X[(size_t)q * nb + bb] *= f;
          x1 *= f;
          x2 *= f;
          xmax *= f;
          sc *= f;
          xv *= f;
        }
        X[(size_t)r * nb + bb] = xv;
        xmax = fmax(xmax, fabs(xv));
        x2 = x1;
        x1 = xv;
      }
      const double inv = xmax > 0.0 ? 1.0 / xmax : 1.0;
      for (int r = 0; r < n; ++r) X[(size_t)r * nb + bb] *= inv;
    }
#undef DL
#undef DG
#undef DU
#undef DU2
#undef PV
    __syncthreads();
    orthonormalize_real(X, n, nb, h, red);
  }
}

hipError_t launch_tridiag_eig(const EigItem *items, int n_items, hipStream_t st) {
  ProfScope ps(K_TRIDIAG, st);
  hipLaunchKernelGGL(tridiag_eig, dim3(n_items), dim3(EIG_THREADS), sizeof(double) * 3 * MAX_N, st, items);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3. Back-transform Y = Q X, Q = H_0 H_1 ... H_{n-2}, H_j = I - tau_j v_j v_j^H.
//    The reflectors of each panel are applied at once in compact WY form,
//    Q_panel = I - V T V^H (T upper triangular, built as in the forward
//    columnwise recurrence T_ii = tau_i, T(0:i, i) = -tau_i T(0:i,0:i) V^H v_i),
//    last panel first.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(EIG_THREADS) backtransform(const EigItem *__restrict__ items) {
  typedef cx<R> C;
  __shared__ C Sm[PANEL][PANEL + 1];
  __shared__ C Tm[PANEL][PANEL + 1];
  __shared__ C W1[PANEL][RR_MAX_BANDS];
  __shared__ C W2[PANEL][RR_MAX_BANDS];
  __shared__ C taus[PANEL];
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N, nb = it.nb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const size_t ld = (size_t)n;
  C *__restrict__ Y = (C *)it.Yb;     // working vectors (== it.Y in FP64)
  const C *__restrict__ A = (const C *)it.A;
  for (size_t e = tid; e < (size_t)n * nb; e += EIG_THREADS) {
    const int r = (int)(e % n), b = (int)(e / n);
    Y[e] = mkc<R>((R)it.X[(size_t)r * nb + b], R(0));
  }
  __syncthreads();
  // v_i[r] of the panel starting at p: 0 above row p+i+1, 1 at it, A below
  auto vent = [&](int p, int i, int r) -> C {
    const int j = p + i;
    if (r <= j) return czero<R>();
    if (r == j + 1) return mkc<R>(R(1), R(0));
    return A[(size_t)j * ld + r];
  };
  const int np = (n - 1 + PANEL - 1) / PANEL;
  for (int pi = np - 1; pi >= 0; --pi) {
    const int p = pi * PANEL;
    const int nbp = min(PANEL, n - 1 - p);
    if (tid < nbp) taus[tid] = ((const C *)it.tau)[p + tid];
    // S(i, k) = v_i^H v_k, i < k
    for (int e = w; e < nbp * nbp; e += EIG_WAVES) {
      const int i = e % nbp, k = e / nbp;
      if (i >= k) continue;
      C acc = czero<R>();
      for (int r = p + k + 1 + lane; r < n; r += 64) acc = cfma_cj(vent(p, i, r), vent(p, k, r), acc);
      acc.re = wave_sum(acc.re);
      acc.im = wave_sum(acc.im);
      if (lane == 0) Sm[i][k] = acc;
    }
    // W1 = V^H Y
    for (int e = w; e < nbp * nb; e += EIG_WAVES) {
      const int i = e % nbp, c = e / nbp;
      C acc = czero<R>();
      for (int r = p + i + 1 + lane; r < n; r += 64) acc = cfma_cj(vent(p, i, r), Y[(size_t)c * ld + r], acc);
      acc.re = wave_sum(acc.re);
      acc.im = wave_sum(acc.im);
      if (lane == 0) W1[i][c] = acc;
    }
    __syncthreads();
    // T by the forward recurrence (small, one wave).  Lane a owns row a of T
    // and only ever reads entries of its own row, so no barrier is needed.
    if (w == 0 && lane < PANEL) {
      for (int i = 0; i < nbp; ++i) {
        C t = czero<R>();
        if (lane < i) {
          for (int b = lane; b < i; ++b) t = cfma(Tm[lane][b], Sm[b][i], t);
          Tm[lane][i] = czero<R>() - taus[i] * t;
        } else if (lane == i) {
          Tm[i][i] = taus[i];
        } else {
          Tm[lane][i] = czero<R>();
        }
      }
    }
    __syncthreads();
    // W2 = T W1
    for (int e = tid; e < nbp * nb; e += EIG_THREADS) {
      const int i = e % nbp, c = e / nbp;
      C acc = czero<R>();
      for (int a = i; a < nbp; ++a) acc = cfma(Tm[i][a], W1[a][c], acc);
      W2[i][c] = acc;
    }
    __syncthreads();
    // Y -= V W2 on rows p+1 .. n-1
    const int rows = n - p - 1;
    for (size_t e = tid; e < (size_t)rows * nb; e += EIG_THREADS) {
      const int r = p + 1 + (int)(e % rows), c = (int)(e / rows);
      const int imax = min(nbp - 1, r - p - 1);
      C acc = czero<R>();
      for (int i = 0; i <= imax; ++i) acc = cfma(vent(p, i, r), W2[i][c], acc);
      C *y = Y + (size_t)c * ld + r;
      *y = *y - acc;
    }
    __syncthreads();
  }
  if (sizeof(R) != sizeof(double)) {
    for (size_t e = tid; e < (size_t)n * nb; e += EIG_THREADS) it.Y[e] = ccast<double>(Y[e]);
  }
}

hipError_t launch_backtransform(const EigItem *items, int n_items, bool fp32, hipStream_t st) {
  ProfScope ps(K_BACKTRANSFORM, st);
  if (fp32)
    hipLaunchKernelGGL(backtransform<float>, dim3(n_items), dim3(EIG_THREADS), 0, st, items);
  else
    hipLaunchKernelGGL(backtransform<double>, dim3(n_items), dim3(EIG_THREADS), 0, st, items);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 4. Rayleigh-Ritz in FP64: orthonormalise Y, G = Y^H C Y, Jacobi
//    eigen-decomposition of G (parallel round-robin ordering), Y <- Y V.
//    Final vectors go to it.Z, eigenvalues to it.lam, frequencies to it.omega.
// ---------------------------------------------------------------------------
constexpr int RR_MAXB = RR_MAX_BANDS;

__device__ void orthonormalize_complex(cd *Y, int n, int nb, cd *h, double *red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const size_t ld = (size_t)n;
  for (int b = 0; b < nb; ++b) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = w; c < b; c += EIG_WAVES) {
        cd acc = mk(0.0, 0.0);
        for (int r = lane; r < n; r += 64) acc = cfma_cj(Y[(size_t)c * ld + r], Y[(size_t)b * ld + r], acc);
        acc.re = wave_sum(acc.re);
        acc.im = wave_sum(acc.im);
        if (lane == 0) h[c] = acc;
      }
      __syncthreads();
      for (int r = tid; r < n; r += EIG_THREADS) {
        cd acc = Y[(size_t)b * ld + r];
        for (int c = 0; c < b; ++c) acc = acc - h[c] * Y[(size_t)c * ld + r];
        Y[(size_t)b * ld + r] = acc;
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int r = tid; r < n; r += EIG_THREADS) s += abs2(Y[(size_t)b * ld + r]);
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int r = tid; r < n; r += EIG_THREADS) Y[(size_t)b * ld + r] = inv * Y[(size_t)b * ld + r];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(EIG_THREADS) rayleigh_ritz(const EigItem *__restrict__ items) {
  __shared__ cd Gs[RR_MAXB][RR_MAXB + 1];
  __shared__ cd Vs[RR_MAXB][RR_MAXB + 1];
  __shared__ cd h[RR_MAXB];
  __shared__ double red[2 * EIG_WAVES];
  __shared__ double rc[RR_MAXB / 2 + 1], rs[RR_MAXB / 2 + 1];
  __shared__ cd rph[RR_MAXB / 2 + 1];
  __shared__ int pa[RR_MAXB / 2 + 1], pb[RR_MAXB / 2 + 1];
  __shared__ int perm[RR_MAXB];
  __shared__ double evs[RR_MAXB];
  __shared__ int active_s;
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N, nb = it.nb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const size_t ld = (size_t)n;
  cd *__restrict__ Y = it.Y;
  cd *__restrict__ Z = it.Z;
  const cd *__restrict__ C = it.Ak;
  orthonormalize_complex(Y, n, nb, h, red);
  // Z = C Y, waves over 64-row strips, 8 columns of Y per pass
  constexpr int NBC = 8;
  const int S = (n + 63) / 64;
  for (int b0 = 0; b0 < nb; b0 += NBC) {
    const int nc = min(NBC, nb - b0);
    for (int s = w; s < S; s += EIG_WAVES) {
      const int r = s * 64 + lane;
      cd acc[NBC];
#pragma unroll
      for (int c = 0; c < NBC; ++c) acc[c] = mk(0.0, 0.0);
      if (r < n) {
        for (int col = 0; col < n; ++col) {
          const cd a = C[(size_t)col * ld + r];
#pragma unroll
          for (int c = 0; c < NBC; ++c)
            if (c < nc) acc[c] = cfma(a, Y[(size_t)(b0 + c) * ld + col], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < NBC; ++c)
          if (c < nc) Z[(size_t)(b0 + c) * ld + r] = acc[c];
      }
    }
  }
  __syncthreads();
  // G = Y^H Z (Hermitian part), V = I
  for (int e = w; e < nb * nb; e += EIG_WAVES) {
    const int a = e % nb, b = e / nb;
    cd acc = mk(0.0, 0.0);
    for (int r = lane; r < n; r += 64) acc = cfma_cj(Y[(size_t)a * ld + r], Z[(size_t)b * ld + r], acc);
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) Gs[a][b] = acc;
  }
  for (int e = tid; e < nb * nb; e += EIG_THREADS) {
    const int a = e % nb, b = e / nb;
    Vs[a][b] = mk(a == b ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += EIG_THREADS) {
    const int a = e % nb, b = e / nb;
    if (a < b) {
      const cd x = Gs[a][b], y2 = Gs[b][a];
      const cd hm = mk(0.5 * (x.re + y2.re), 0.5 * (x.im - y2.im));
      Gs[a][b] = hm;
      Gs[b][a] = conj(hm);
    } else if (a == b) {
      Gs[a][a].im = 0.0;
    }
  }
  __syncthreads();
  // parallel cyclic Jacobi, round-robin pairing over nbe (even) indices
  const int nbe = nb + (nb & 1);
  const int npair = nbe / 2;
  double fro = 0.0;
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) fro += abs2(Gs[a][b]);
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b)
        if (a != b) off += abs2(Gs[a][b]);
    if (off <= 1e-34 * fro) break;
    for (int round = 0; round < nbe - 1; ++round) {
      if (tid < npair) {
        // round-robin: index 0 fixed, others rotate
        int i1, i2;
        if (tid == 0) { i1 = 0; i2 = 1 + (round % (nbe - 1)); }
        else {
          i1 = 1 + ((round + tid) % (nbe - 1));
          i2 = 1 + ((round + nbe - 1 - tid) % (nbe - 1));
        }
        int pp = min(i1, i2), qq = max(i1, i2);
        double c = 1.0, s = 0.0;
        cd ph = mk(1.0, 0.0);
        if (qq < nb) {
          const cd gpq = Gs[pp][qq];
          const double ab = sqrt(abs2(gpq));
          if (ab > 1e-300 && ab * ab > 1e-36 * fabs(Gs[pp][pp].re * Gs[qq][qq].re) ) {
            ph = mk(gpq.re / ab, -gpq.im / ab);  // e^{-i phi}
            const double zeta = (Gs[qq][qq].re - Gs[pp][pp].re) / (2.0 * ab);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = c * t;
          }
        } else {
          qq = pp;  // dummy partner
        }
        pa[tid] = pp;
        pb[tid] = qq;
        rc[tid] = c;
        rs[tid] = s;
        rph[tid] = ph;
      }
      __syncthreads();
      // columns: G J and V J, J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
      for (int e = tid; e < npair * nb; e += EIG_THREADS) {
        const int k = e / nb, row = e % nb;
        const int pp = pa[k], qq = pb[k];
        if (pp == qq || rs[k] == 0.0) continue;
        const double c = rc[k], s = rs[k];
        const cd ph = rph[k];
        const cd gp = Gs[row][pp], gq = Gs[row][qq];
        Gs[row][pp] = c * gp - s * (ph * gq);
        Gs[row][qq] = s * gp + c * (ph * gq);
        const cd vp = Vs[row][pp], vq = Vs[row][qq];
        Vs[row][pp] = c * vp - s * (ph * vq);
        Vs[row][qq] = s * vp + c * (ph * vq);
      }
      __syncthreads();
      // rows: J^H (G J)
      for (int e = tid; e < npair * nb; e += EIG_THREADS) {
        const int k = e / nb, col = e % nb;
        const int pp = pa[k], qq = pb[k];
        if (pp == qq || rs[k] == 0.0) continue;
        const double c = rc[k], s = rs[k];
        const cd phc = conj(rph[k]);
        const cd gp = Gs[pp][col], gq = Gs[qq][col];
        Gs[pp][col] = c * gp - s * (phc * gq);
        Gs[qq][col] = s * gp + c * (phc * gq);
      }
      __syncthreads();
    }
  }
  // sort eigenvalues ascending
  if (tid == 0) {
    for (int a = 0; a < nb; ++a) { perm[a] = a; evs[a] = Gs[a][a].re; }
    for (int a = 0; a < nb; ++a) {
      int best = a;
      for (int b = a + 1; b < nb; ++b)
        if (evs[perm[b]] < evs[perm[best]]) best = b;
      const int t = perm[a]; perm[a] = perm[best]; perm[best] = t;
    }
  }
  __syncthreads();
  if (tid < nb) {
    const double lam = evs[perm[tid]];
    it.lam[tid] = lam;
    it.omega[tid] = sqrt(fmax(lam, 0.0));
  }
  // Z = Y V(:, perm)
  for (size_t e = tid; e < (size_t)n * nb; e += EIG_THREADS) {
    const int r = (int)(e % n), b = (int)(e / n);
    const int pbb = perm[b];
    cd acc = mk(0.0, 0.0);
    for (int a = 0; a < nb; ++a) acc = cfma(Y[(size_t)a * ld + r], Vs[a][pbb], acc);
    Z[(size_t)b * ld + r] = acc;
  }
  (void)active_s;
}

hipError_t launch_rayleigh_ritz(const EigItem *items, int n_items, hipStream_t st) {
  ProfScope ps(K_RR, st);
  hipLaunchKernelGGL(rayleigh_ritz, dim3(n_items), dim3(EIG_THREADS), 0, st, items);
  return hipGetLastError();
}

// Dynamic LDS above the default limit has to be opted into per kernel.
hipError_t init_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute((const void *)hetrd_panel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(cd) * 2 * MAX_N));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)hetrd_panel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(cf) * 2 * MAX_N));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)tridiag_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * 3 * MAX_N));
}

}  // namespace mvpb
