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

// ---------------------------------------------------------------------------
// 1a. Panel kernel: columns p .. p+nbp-1 of every item.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(EIG_THREADS) hetrd_panel(const EigItem *__restrict__ items, int p) {
  extern __shared__ cd sh[];
  cd *v = sh;                  // MAX_N: current reflector (rows j+1..n-1)
  cd *y = v + MAX_N;           // MAX_N: new column of W
  cd *part = y + MAX_N;        // 1024: matrix-vector partial sums
  __shared__ double red[2 * EIG_WAVES];
  __shared__ cd t1[PANEL], t2[PANEL], wj[PANEL], vj[PANEL];
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N;
  if (p >= n - 1) return;
  const int nbp = min(PANEL, n - 1 - p);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  cd *__restrict__ A = it.A;
  cd *__restrict__ W = it.W;
  const size_t ld = (size_t)n;

  for (int i = 0; i < nbp; ++i) {
    const int j = p + i;
    // --- step 1: bring column j up to date with the panel's earlier reflectors
    if (tid < i) {
      wj[tid] = conj(W[(size_t)tid * ld + j]);
      vj[tid] = conj(A[(size_t)(p + tid) * ld + j]);
    }
    __syncthreads();
    for (int r = j + tid; r < n; r += EIG_THREADS) {
      cd acc = A[(size_t)j * ld + r];
      for (int k = 0; k < i; ++k) {
        acc = acc - A[(size_t)(p + k) * ld + r] * wj[k];
        acc = acc - W[(size_t)k * ld + r] * vj[k];
      }
      if (r == j) acc.im = 0.0;
      A[(size_t)j * ld + r] = acc;
    }
    __syncthreads();
    // --- step 2: reflector annihilating A[j+2:n, j]
    double xn2 = 0.0;
    for (int r = j + 2 + tid; r < n; r += EIG_THREADS) xn2 += abs2(A[(size_t)j * ld + r]);
    xn2 = block_sum(xn2, red);
    const cd alpha = A[(size_t)j * ld + j + 1];
    cd tau = mk(0.0, 0.0), scale = mk(0.0, 0.0);
    double beta = alpha.re;
    if (!(xn2 == 0.0 && alpha.im == 0.0)) {
      const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
      beta = alpha.re >= 0.0 ? -nrm : nrm;
      tau = mk((beta - alpha.re) / beta, -alpha.im / beta);
      scale = cdiv(mk(1.0, 0.0), alpha - mk(beta, 0.0));
    }
    const int m = n - j - 1;
    for (int r = j + 1 + tid; r < n; r += EIG_THREADS) {
      cd x;
      if (r == j + 1) {
        x = mk(1.0, 0.0);
      } else {
        x = A[(size_t)j * ld + r] * scale;
      }
      A[(size_t)j * ld + r] = x;
      v[r - j - 1] = x;
    }
    if (tid == 0) {
      it.d[j] = A[(size_t)j * ld + j].re;
      it.e[j] = beta;
      it.tau[j] = tau;
    }
    __syncthreads();
    // --- step 3: y = A22 v with A22 = A[j+1:, j+1:] (pre-panel values)
    const cd *A22 = A + (size_t)(j + 1) * ld + (j + 1);
    const int S = (m + 63) / 64;
    if (S >= EIG_WAVES) {
      for (int s = w; s < S; s += EIG_WAVES) {
        const int r = s * 64 + lane;
        if (r < m) {
          cd a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0);
          int c = 0;
          for (; c + 1 < m; c += 2) {
            a0 = cfma(A22[(size_t)c * ld + r], v[c], a0);
            a1 = cfma(A22[(size_t)(c + 1) * ld + r], v[c + 1], a1);
          }
          if (c < m) a0 = cfma(A22[(size_t)c * ld + r], v[c], a0);
          y[r] = a0 + a1;
        }
      }
    } else {
      const int G = EIG_WAVES / S;
      const int s = w % S, g = w / S;
      if (g < G) {
        const int c0 = (int)((long)g * m / G), c1 = (int)((long)(g + 1) * m / G);
        const int r = s * 64 + lane;
        cd a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0);
        if (r < m) {
          int c = c0;
          for (; c + 1 < c1; c += 2) {
            a0 = cfma(A22[(size_t)c * ld + r], v[c], a0);
            a1 = cfma(A22[(size_t)(c + 1) * ld + r], v[c + 1], a1);
          }
          if (c < c1) a0 = cfma(A22[(size_t)c * ld + r], v[c], a0);
        }
        part[g * S * 64 + s * 64 + lane] = a0 + a1;
      }
      __syncthreads();
      for (int r = tid; r < m; r += EIG_THREADS) {
        cd acc = mk(0.0, 0.0);
        for (int gg = 0; gg < G; ++gg) acc = acc + part[gg * S * 64 + r];
        y[r] = acc;
      }
    }
    __syncthreads();
    // corrections with the panel's earlier columns (V = A[:, p:p+i], W[:, 0:i])
    if (i > 0) {
      for (int k = w; k < 2 * i; k += EIG_WAVES) {
        const bool isW = k < i;
        const int kk = isW ? k : k - i;
        const cd *col = isW ? (W + (size_t)kk * ld) : (A + (size_t)(p + kk) * ld);
        cd acc = mk(0.0, 0.0);
        for (int r = j + 1 + lane; r < n; r += 64) acc = cfma_cj(col[r], v[r - j - 1], acc);
        acc.re = wave_sum(acc.re);
        acc.im = wave_sum(acc.im);
        if (lane == 0) {
          if (isW) t1[kk] = acc; else t2[kk] = acc;
        }
      }
      __syncthreads();
      for (int r = j + 1 + tid; r < n; r += EIG_THREADS) {
        cd acc = y[r - j - 1];
        for (int k = 0; k < i; ++k) {
          acc = acc - A[(size_t)(p + k) * ld + r] * t1[k];
          acc = acc - W[(size_t)k * ld + r] * t2[k];
        }
        y[r - j - 1] = acc;
      }
      __syncthreads();
    }
    // y = tau y ; y += (-1/2 tau (y^H v)) v
    cd dot = mk(0.0, 0.0);
    for (int r = tid; r < m; r += EIG_THREADS) {
      const cd yy = tau * y[r];
      y[r] = yy;
      dot = cfma_cj(yy, v[r], dot);
    }
    dot = block_sum_c(dot, red);
    const cd al2 = mk(-0.5, 0.0) * tau * dot;
    for (int r = tid; r < m; r += EIG_THREADS) {
      const cd yy = cfma(al2, v[r], y[r]);
      W[(size_t)i * ld + j + 1 + r] = yy;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 1b. Trailing update A[q0:, q0:] -= V W^H + W V^H, q0 = p + nbp (full square).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) hetrd_update(const EigItem *__restrict__ items, int p) {
  constexpr int BK = 8;
  __shared__ cd Vr[BK][65], Wr[BK][65], Vc[BK][65], Wc[BK][65];
  const EigItem it = items[blockIdx.z];
  const int n = 2 * it.N;
  if (p >= n - 1) return;
  const int nbp = min(PANEL, n - 1 - p);
  const int q0 = p + nbp, m = n - q0;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (r0 >= m || c0 >= m) return;
  cd *__restrict__ A = it.A;
  const cd *__restrict__ W = it.W;
  const size_t ld = (size_t)n;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  cd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = mk(0.0, 0.0);
  for (int k0 = 0; k0 < nbp; k0 += BK) {
    for (int e = tid; e < 64 * BK; e += 256) {
      const int i = e & 63, k = e >> 6;
      const int gk = k0 + k;
      const int gr = q0 + r0 + i, gc = q0 + c0 + i;
      cd vr = mk(0.0, 0.0), wr = vr, vc = vr, wc = vr;
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
      cd a1[4], a2[4], b1[4], b2[4];
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
      cd *dst = A + (size_t)gc * ld + gr;
      *dst = *dst - acc[a][b];
    }
  }
}

hipError_t launch_hetrd(const EigItem *items, int n_items, int n_max, hipStream_t st) {
  const size_t sh = sizeof(cd) * (2 * MAX_N + 1024);
  for (int p = 0; p < n_max - 1; p += PANEL) {
    {
      ProfScope ps(K_HETRD_PANEL, st);
      hipLaunchKernelGGL(hetrd_panel, dim3(n_items), dim3(EIG_THREADS), sh, st, items, p);
    }
    const int nbp = min(PANEL, n_max - 1 - p);
    const int m = n_max - p - nbp;
    if (m > 0) {
      const int t = (m + 63) / 64;
      ProfScope ps(K_HETRD_UPDATE, st);
      hipLaunchKernelGGL(hetrd_update, dim3(t, t, n_items), dim3(256), 0, st, items, p);
    }
  }
  return hipGetLastError();
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
  double *ee2 = dd + MAX_N;    // MAX_N
  __shared__ double lo[64], hi[64], xs[EIG_THREADS];
  __shared__ int cnts[EIG_THREADS];
  __shared__ double red[2 * EIG_WAVES];
  __shared__ double h[64];
  __shared__ int done_s;
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N, nb = it.nb;
  const int tid = threadIdx.x;
  if (tid == 0) it.d[n - 1] = it.A[(size_t)(n - 1) * n + (n - 1)].re;
  // stage d, e^2; Gershgorin bounds
  double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
  for (int r = tid; r < n; r += EIG_THREADS) {
    const double dr = (r == n - 1) ? it.A[(size_t)(n - 1) * n + (n - 1)].re : it.d[r];
    const double er = (r < n - 1) ? it.e[r] : 0.0;
    const double el = (r > 0) ? it.e[r - 1] : 0.0;
    dd[r] = dr;
    if (r < n - 1) ee2[r] = er * er;
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
    for (int r = 0; r < n; ++r) {
      DG(r) = dd[r] - lam;
      if (r < n - 1) {
        const double er = it.e[r];
        DL(r) = er;
        DU(r) = er;
      }
    }
    // LU with partial pivoting of the tridiagonal T - lam I
    for (int r = 0; r < n - 1; ++r) {
      const double dr = DG(r), lr = DL(r);
      if (fabs(dr) >= fabs(lr)) {
        const double piv = (dr == 0.0) ? pert : dr;
        DG(r) = piv;
        const double f = lr / piv;
        DL(r) = f;
        DG(r + 1) = DG(r + 1) - f * DU(r);
        if (r < n - 2) DU2(r) = 0.0;
        PV(r) = 0.0;
      } else {
        const double f = dr / lr;
        DG(r) = lr;
        DL(r) = f;
        const double tmp = DU(r);
        DU(r) = DG(r + 1);
        DG(r + 1) = tmp - f * DG(r + 1);
        if (r < n - 2) {
          DU2(r) = DU(r + 1);
          DU(r + 1) = -f * DU(r + 1);
        }
        PV(r) = 1.0;
      }
    }
    if (DG(n - 1) == 0.0) DG(n - 1) = pert;
    for (int r = 0; r < n; ++r) X[(size_t)r * nb + bb] = hash_uniform(r + 1, bb + 7);
  }
  for (int iter = 0; iter < 3; ++iter) {
    if (tid < nb) {
      const int bb = tid;
      // forward: apply P and L^-1
      for (int r = 0; r < n - 1; ++r) {
        double xr = X[(size_t)r * nb + bb], xr1 = X[(size_t)(r + 1) * nb + bb];
        if (PV(r) != 0.0) { const double t = xr; xr = xr1; xr1 = t; X[(size_t)r * nb + bb] = xr; }
        X[(size_t)(r + 1) * nb + bb] = xr1 - DL(r) * xr;
      }
      // back substitution with U (diag, super, super-super), scaled to avoid overflow
      double xmax = 0.0;
      for (int r = n - 1; r >= 0; --r) {
        double s = X[(size_t)r * nb + bb];
        if (r + 1 < n) s -= DU(r) * X[(size_t)(r + 1) * nb + bb];
        if (r + 2 < n) s -= DU2(r) * X[(size_t)(r + 2) * nb + bb];
        double xv = s / DG(r);
        if (!isfinite(xv)) xv = 0.0;
        X[(size_t)r * nb + bb] = xv;
        xmax = fmax(xmax, fabs(xv));
        if (xmax > 1e150) {
          // rescale the solved tail to keep it finite
          const double sc = 1.0 / xmax;
          for (int q = r; q < n; ++q) X[(size_t)q * nb + bb] *= sc;
          xmax = 1.0;
          // unsolved head is scaled as well so the system stays consistent
          for (int q = 0; q < r; ++q) X[(size_t)q * nb + bb] *= sc;
        }
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
  hipLaunchKernelGGL(tridiag_eig, dim3(n_items), dim3(EIG_THREADS), sizeof(double) * 2 * MAX_N, st, items);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3. Back-transform Y = Q X, Q = H_0 H_1 ... H_{n-2}, H_j = I - tau_j v_j v_j^H.
//    Each wave owns a set of columns, so no block-wide barrier is needed.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(EIG_THREADS) backtransform(const EigItem *__restrict__ items) {
  const EigItem it = items[blockIdx.x];
  const int n = 2 * it.N, nb = it.nb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const size_t ld = (size_t)n;
  cd *__restrict__ Y = it.Y;
  const cd *__restrict__ A = it.A;
  for (size_t e = tid; e < (size_t)n * nb; e += EIG_THREADS) {
    const int r = (int)(e % n), b = (int)(e / n);
    Y[e] = mk(it.X[(size_t)r * nb + b], 0.0);
  }
  __syncthreads();
  constexpr int CPW = 4;  // columns per wave pass
  for (int b0 = w * CPW; b0 < nb; b0 += EIG_WAVES * CPW) {
    const int ncol = min(CPW, nb - b0);
    for (int j = n - 2; j >= 0; --j) {
      const cd tau = it.tau[j];
      if (tau.re == 0.0 && tau.im == 0.0) continue;
      cd s[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) s[c] = mk(0.0, 0.0);
      for (int r = j + 1 + lane; r < n; r += 64) {
        const cd vr = (r == j + 1) ? mk(1.0, 0.0) : A[(size_t)j * ld + r];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
          if (c < ncol) s[c] = cfma_cj(vr, Y[(size_t)(b0 + c) * ld + r], s[c]);
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        s[c].re = wave_sum(s[c].re);
        s[c].im = wave_sum(s[c].im);
        s[c] = tau * s[c];
      }
      for (int r = j + 1 + lane; r < n; r += 64) {
        const cd vr = (r == j + 1) ? mk(1.0, 0.0) : A[(size_t)j * ld + r];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
          if (c < ncol) {
            cd *y = Y + (size_t)(b0 + c) * ld + r;
            *y = *y - vr * s[c];
          }
      }
    }
  }
}

hipError_t launch_backtransform(const EigItem *items, int n_items, hipStream_t st) {
  ProfScope ps(K_BACKTRANSFORM, st);
  hipLaunchKernelGGL(backtransform, dim3(n_items), dim3(EIG_THREADS), 0, st, items);
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
  hipError_t e = hipFuncSetAttribute((const void *)hetrd_panel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(cd) * (2 * MAX_N + 1024)));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)tridiag_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * 2 * MAX_N));
}

}  // namespace mvpb
