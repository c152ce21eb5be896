// Tridiagonal eigenpairs and the FP64 Rayleigh-Ritz refinement of the
// batched Hermitian eigensolve (the reductions live in band.hip).
//  1. Lowest nb eigenvalues of T by multisection on Sturm counts; their
//     eigenvectors by inverse iteration with a pivoted tridiagonal LU,
//     re-orthonormalised as a block after each sweep.
//  2. FP64 Rayleigh-Ritz on span(Y) with the kept copy of C(k):
//     eigenpairs of Y^H C Y, omega = sqrt(max(lambda, 0)).
#include <float.h>

#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

constexpr int EIG_THREADS = 1024;
constexpr int EIG_WAVES = EIG_THREADS / 64;

// ---------------------------------------------------------------------------
// 1. Tridiagonal eigenproblem: multisection for the lowest nb eigenvalues,
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
// 2. Rayleigh-Ritz in FP64: orthonormalise Y, G = Y^H C Y, Jacobi
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
  hipError_t e = hipFuncSetAttribute((const void *)tridiag_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(double) * 3 * MAX_N));
  if (e != hipSuccess) return e;
  return init_band_attributes();
}

}  // namespace mvpb
