// General compliance and three-dimensional cells: the reduced operator of
// eq. (eigenvalueproblem) built from the full stress-space compliance matrix
// Phi instead of the isotropic block form.
//
// Unknowns: d = 2 (planar) or 3 (spatial) displacement components of N plane
// waves, n_s = 3 or 6 Voigt stress components (planar 11, 22, 12; spatial 11,
// 22, 33, 23, 13, 12).  With exact subdomain integrals (J = |Omega| I) the
// coupling of Sec. 4.1 eq. (eh) (and its spatial form of Sec. 2.3) is
// H = i |Omega| H', where H' has the blocks diag(K_b) at (u_a, sigma_(ab)) and
// diag(K_a) at (u_b, sigma_(ab)) for a != b, K_l = G_l + kappa_l per plane
// wave.  With Phi = L_P L_P^H and Omega = I_d (x) L_R L_R^H, the standard
// form C(k) = (I (x) L_R^-1) H Phi^-1 H^H (I (x) L_R^-H) = |Omega|^2 Z Z^H,
// Z = (I (x) L_R^-1) H' L_P^-H = Z_0 + sum_l kappa_l Z_l, so
//   C(k) = |Omega|^2 sum_{l <= m} kappa_l kappa_m C_lm   (kappa_0 = 1),
//   C_ll = Z_l Z_l^H,  C_lm = Z_l Z_m^H + Z_m Z_l^H (l < m),
// (d+1)(d+2)/2 Hermitian n x n coefficient matrices per cell, n = d N.
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

// exp(i pi num / den), num reduced modulo 2 den first (exact argument reduction)
MVPB_DEV cd expipi(long num, int den) {
  long t = num % (2L * den);
  if (t < 0) t += 2L * den;
  double s, c;
  sincospi((double)t / (double)den, &s, &c);
  return mk(c, s);
}

MVPB_DEV double sinc_pi(int m, int n) {
  return m == 0 ? 1.0 : sinpi((double)m / n) / (M_PI * (double)m / n);
}

// ---------------------------------------------------------------------------
// Structure factors of every weight field f on the difference grid,
//   F_f(m, q, r) = sum over voxels (i, j, k) of w_f(phase(i, j, k))
//                  |Omega|/(nx ny nz) e^{i 2 pi (m (i+1/2)/nx + q (j+1/2)/ny + r (k+1/2)/nz)}
//                  sinc(m/nx) sinc(q/ny) sinc(r/nz),
// (the exact integral of e^{i dG . x} over each voxel, Sec. 3 / Sec. 4.1),
// contracted one axis at a time (k, then j, then i) in FP64.  A planar pixel
// cell is the case nz = 1, M3 = 0.  Phase map [nx][ny][nz], weights [P][nf].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) sf_gen_pass_z(const int32_t *__restrict__ phase, const double *__restrict__ gw,
                                                     int nf, int nx, int ny, int nz, int M3, cd *__restrict__ X1) {
  const int nr = 4 * M3 + 1;
  const size_t total = (size_t)nf * nx * ny * nr;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int r = (int)(e % nr);
  const size_t ij = (e / nr) % ((size_t)nx * ny);
  const int f = (int)(e / nr / ((size_t)nx * ny));
  const int rr = r - 2 * M3;
  cd acc = mk(0.0, 0.0);
  const int32_t *ph = phase + ij * nz;
  for (int k = 0; k < nz; ++k) acc = acc + gw[(size_t)ph[k] * nf + f] * expipi((long)rr * (2 * k + 1), nz);
  X1[e] = acc;   // [f][i][j][r]
}

__global__ void __launch_bounds__(256) sf_gen_pass_y(const cd *__restrict__ X1, int nf, int nx, int ny, int nr, int M2,
                                                     cd *__restrict__ X2) {
  const int nq = 4 * M2 + 1;
  const size_t total = (size_t)nf * nx * nq * nr;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int r = (int)(e % nr);
  const int q = (int)((e / nr) % nq);
  const size_t fi = e / nr / nq;   // f * nx + i
  const int qq = q - 2 * M2;
  cd acc = mk(0.0, 0.0);
  const cd *x = X1 + fi * (size_t)ny * nr + r;
  for (int j = 0; j < ny; ++j) acc = acc + x[(size_t)j * nr] * expipi((long)qq * (2 * j + 1), ny);
  X2[e] = acc;   // [f][i][q][r]
}

__global__ void __launch_bounds__(256) sf_gen_pass_x(const cd *__restrict__ X2, int nf, int nx, int ny, int nz, int M1,
                                                     int M2, int M3, double vol, cd *__restrict__ F) {
  const int nm = 4 * M1 + 1, nq = 4 * M2 + 1, nr = 4 * M3 + 1;
  const size_t total = (size_t)nf * nm * nq * nr;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const size_t qr = e % ((size_t)nq * nr);
  const int m = (int)((e / ((size_t)nq * nr)) % nm);
  const int f = (int)(e / ((size_t)nq * nr) / nm);
  const int q = (int)(qr / nr), r = (int)(qr % nr);
  const int mm = m - 2 * M1, qq = q - 2 * M2, rr = r - 2 * M3;
  cd acc = mk(0.0, 0.0);
  const cd *x = X2 + (size_t)f * nx * nq * nr + qr;
  for (int i = 0; i < nx; ++i) acc = acc + x[(size_t)i * nq * nr] * expipi((long)mm * (2 * i + 1), nx);
  const double sc = vol / ((double)nx * ny * nz) * sinc_pi(mm, nx) * sinc_pi(qq, ny) * sinc_pi(rr, nz);
  F[e] = sc * acc;   // [f][m][q][r]
}

hipError_t launch_structure_factors_general(const int32_t *phase, const double *gw, int nf, int nx, int ny, int nz,
                                            int M1, int M2, int M3, double vol, cd *X1, cd *X2, cd *F,
                                            hipStream_t st) {
  const int nm = 4 * M1 + 1, nq = 4 * M2 + 1, nr = 4 * M3 + 1;
  const size_t t1 = (size_t)nf * nx * ny * nr, t2 = (size_t)nf * nx * nq * nr, t3 = (size_t)nf * nm * nq * nr;
  ProfScope ps(K_SF, st);
  hipLaunchKernelGGL(sf_gen_pass_z, dim3((unsigned)((t1 + 255) / 256)), dim3(256), 0, st, phase, gw, nf, nx, ny, nz,
                     M3, X1);
  hipLaunchKernelGGL(sf_gen_pass_y, dim3((unsigned)((t2 + 255) / 256)), dim3(256), 0, st, X1, nf, nx, ny, nr, M2, X2);
  hipLaunchKernelGGL(sf_gen_pass_x, dim3((unsigned)((t3 + 255) / 256)), dim3(256), 0, st, X2, nf, nx, ny, nz, M1, M2,
                     M3, vol, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block-Toeplitz scatter: out[(s N + r), (t N + c)] = F_{fmap[s][t]}(n_c - n_r)
// (Sec. 4.1 eqs. (eo), (ep): every entry is the integral of the weight times
// e^{i (K_c - K_r) . x}, i.e. the difference-grid table at n_c - n_r; row =
// test function r, column = trial function c).  Column-major, leading
// dimension nblk N.  Plane wave r = ((a + M1)(2M2+1) + (b + M2))(2M3+1) + (c + M3).
// ---------------------------------------------------------------------------
struct BlockMap {
  int f[36];
};

MVPB_DEV void pw_index(int r, int M2, int M3, int *a, int *b, int *c) {
  const int n3 = 2 * M3 + 1, n2 = 2 * M2 + 1;
  *c = r % n3;
  *b = (r / n3) % n2;
  *a = r / n3 / n2;
}

__global__ void __launch_bounds__(256) toeplitz_blocks(const cd *__restrict__ F, int M1, int M2, int M3, int N,
                                                       int nblk, BlockMap map, cd *__restrict__ out) {
  const int nq = 4 * M2 + 1, nr = 4 * M3 + 1, nm = 4 * M1 + 1;
  const int ld = nblk * N;
  const int row = blockIdx.x * 256 + threadIdx.x;
  const int col = blockIdx.y;
  if (row >= ld) return;
  const int s = row / N, r = row % N, t = col / N, c = col % N;
  int ra, rb, rc, ca, cb, cc;
  pw_index(r, M2, M3, &ra, &rb, &rc);
  pw_index(c, M2, M3, &ca, &cb, &cc);
  const size_t tab = ((size_t)(ca - ra + 2 * M1) * nq + (cb - rb + 2 * M2)) * nr + (cc - rc + 2 * M3);
  out[(size_t)col * ld + row] = F[(size_t)map.f[s * nblk + t] * nm * nq * nr + tab];
}

hipError_t launch_toeplitz_blocks(const cd *F, int M1, int M2, int M3, int N, int nblk, const int *fmap, cd *out,
                                  hipStream_t st) {
  BlockMap m{};
  for (int i = 0; i < nblk * nblk; ++i) m.f[i] = fmap[i];
  const int ld = nblk * N;
  ProfScope ps(K_SCATTER, st);
  hipLaunchKernelGGL(toeplitz_blocks, dim3((ld + 255) / 256, ld), dim3(256), 0, st, F, M1, M2, M3, N, nblk, m, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// C(k) of every general-layout item: lower 32 x 32 tiles computed from the
// coefficient matrices (index of the pair l <= m: l (d+1) - l (l-1)/2 + m - l),
// written to A (reduction precision, lower triangle) and to the kept FP64 copy
// (both triangles).
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) form_operator_general(const EigItem *__restrict__ items) {
  __shared__ cd tile[32][33];
  const EigItem &it = items[blockIdx.x];   // item fastest (coefficient tiles shared in L2)
  if (it.dim == 0) return;   // isotropic planar layout: form_operator
  const int n = it.n, d = it.dim;
  const int nt = (n + 31) / 32;
  int t = blockIdx.y;
  if (t >= nt * (nt + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const double kap[4] = {1.0, it.kap1, it.kap2, it.kap3};
  double w[10];
  int nc = 0;
  for (int l = 0; l <= d; ++l)
    for (int m = l; m <= d; ++m) w[nc++] = kap[l] * kap[m];
  const size_t nn = (size_t)n * n;
  const cd *cf = it.coef;
  const int lr = threadIdx.x & 31, lc0 = threadIdx.x >> 5;
  for (int lc = lc0; lc < 32; lc += 8) {
    const int r = I * 32 + lr, c = J * 32 + lc;
    cd v = mk(0.0, 0.0);
    if (r < n && c < n && r >= c) {
      const size_t e = (size_t)c * n + r;
      for (int q = 0; q < nc; ++q) v = v + w[q] * gld(cf, q * nn + e);
      if (r == c) v.im = 0.0;
      ((cx<R> *)it.A)[e] = ccast<R>(v);
      it.Ak[e] = v;
    }
    tile[lc][lr] = v;
  }
  __syncthreads();
  for (int lc = lc0; lc < 32; lc += 8) {
    const int r = J * 32 + lr, c = I * 32 + lc;
    if (r < n && c < n && r < c) {
      it.Ak[(size_t)c * n + r] = conj(tile[lr][lc]);   // the working copy keeps its lower triangle only
    }
  }
}

hipError_t launch_form_operator_general(const EigItem *items, int n_items, int n_max, bool fp32, hipStream_t st) {
  const int nt = (n_max + 31) / 32;
  const int tiles = nt * (nt + 1) / 2;
  ProfScope ps(K_FORM, st);
  if (fp32)
    hipLaunchKernelGGL((form_operator_general<float>), dim3(n_items, tiles), dim3(256), 0, st, items);
  else
    hipLaunchKernelGGL((form_operator_general<double>), dim3(n_items, tiles), dim3(256), 0, st, items);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Right-hand sides of the stress modes S = -Phi^-1 H* U (Sec. 3, after eq.
// (eigenvalueproblem)): X = H* U with H* = -H^T, i.e. for the Voigt component
// s = (a, b):  X_s = -i |Omega| (K_b o U_a + [a != b] K_a o U_b),
// K_l = 2 pi (T (Q + n))_l per plane wave.  U [n_k][nb][d N], X [n_k][nb][n_s N]
// (per point an (n_s N) x nb column-major block).  Q [n_k][d] on the device.
// ---------------------------------------------------------------------------
struct Tmat {
  double t[9];
};

MVPB_DEV void voigt_pair(int d, int s, int *a, int *b) {
  if (d == 2) {
    const int A[3] = {0, 1, 0}, B[3] = {0, 1, 1};
    *a = A[s];
    *b = B[s];
  } else {
    const int A[6] = {0, 1, 2, 1, 0, 0}, B[6] = {0, 1, 2, 2, 2, 1};
    *a = A[s];
    *b = B[s];
  }
}

__global__ void __launch_bounds__(256) stress_rhs_general(const cd *__restrict__ U, const double *__restrict__ Q,
                                                          int n_k, int nb, int d, int M1, int M2, int M3, Tmat T,
                                                          double vol, cd *__restrict__ X) {
  const int N = (2 * M1 + 1) * (2 * M2 + 1) * (2 * M3 + 1);
  const int ns = d == 2 ? 3 : 6;
  const size_t per = (size_t)ns * N;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per * nb * n_k) return;
  const int row = (int)(e % per);
  const size_t tb = e / per;   // t * nb + band
  const int t = (int)(tb / nb);
  const int s = row / N, i = row % N;
  int a, b, na, nbb, nc;
  voigt_pair(d, s, &a, &b);
  pw_index(i, M2, M3, &na, &nbb, &nc);
  const double qn[3] = {Q[(size_t)t * d] + (na - M1), Q[(size_t)t * d + 1] + (nbb - M2),
                        d == 3 ? Q[(size_t)t * d + 2] + (nc - M3) : 0.0};
  double K[3];
  for (int l = 0; l < d; ++l) {
    double acc = 0.0;
    for (int j = 0; j < d; ++j) acc += T.t[l * d + j] * qn[j];
    K[l] = 2.0 * M_PI * acc;
  }
  const cd *u = U + tb * (size_t)d * N;
  cd v = K[b] * u[(size_t)a * N + i];
  if (a != b) v = v + K[a] * u[(size_t)b * N + i];
  // -i |Omega| v
  X[e] = mk(vol * v.im, -vol * v.re);
}

hipError_t launch_stress_rhs_general(const cd *U, const double *Q, int n_k, int nb, int d, int M1, int M2, int M3,
                                     const double *T, double vol, cd *X, hipStream_t st) {
  Tmat tm{};
  for (int i = 0; i < d * d; ++i) tm.t[i] = T[i];
  const int N = (2 * M1 + 1) * (2 * M2 + 1) * (2 * M3 + 1);
  const size_t total = (size_t)(d == 2 ? 3 : 6) * N * nb * n_k;
  hipLaunchKernelGGL(stress_rhs_general, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U, Q, n_k, nb, d,
                     M1, M2, M3, tm, vol, X);
  return hipGetLastError();
}

}  // namespace mvpb
