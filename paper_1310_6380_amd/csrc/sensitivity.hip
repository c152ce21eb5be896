// Eigenvalue sensitivities with respect to the material of every pixel or
// voxel, for gradient-based band-structure design.
//
// Differentiating A U = lambda Omega U (Sec. 3, eq. (eigenvalueproblem),
// A = H Phi^-1 H*, U^H Omega U = 1) at a simple eigenvalue gives
//   d lambda = -S^H dPhi S - lambda U^H dOmega U,   S = -Phi^-1 H* U.
// The weight w_st of cell element p (an entry of its engineering-Voigt
// compliance, the Phi weights of Sec. 4.1 eq. (ep)) enters Phi through the
// element's Toeplitz block T_p[r, c] = I_p(n_c - n_r) in the blocks (s, t) and
// (t, s); its density enters Omega through I_d (x) T_p (eq. (eo)).  Hence
//   S_s^H T_p S_t = sum_D I_p(D) c_st(D),  c_st(D) = sum_r conj(S_s[r]) S_t[r + D],
// a correlation of the two coefficient vectors on the difference grid
// followed by the exact element integral I_p(D) of e^{i D . x}, which for all
// elements at once is the adjoint of the structure-factor contraction:
//   g(i, j, k) = |Omega|/(nx ny nz) sum_{m,q,r} sinc(m/nx) sinc(q/ny) sinc(r/nz) c(m, q, r)
//                e^{i 2 pi (m (i+1/2)/nx + q (j+1/2)/ny + r (k+1/2)/nz)}.
// d lambda / d w_ss = -Re g_ss, d lambda / d w_st = -2 Re g_st (s < t, both
// blocks), d lambda / d rho = -lambda Re g_rho with c_rho = sum_a (U_a, U_a).
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

namespace {

MVPB_DEV cd eipi(long num, int den) {   // exp(i pi num / den), exact reduction mod 2 den
  long t = num % (2L * den);
  if (t < 0) t += 2L * den;
  double s, c;
  sincospi((double)t / (double)den, &s, &c);
  return mk(c, s);
}

MVPB_DEV double sincp(int m, int n) { return m == 0 ? 1.0 : sinpi((double)m / n) / (M_PI * (double)m / n); }

}  // namespace

// C[item][f][D]: correlations of the stress components (pairs s <= t, upper
// triangle row by row) and of the displacement (last field) of one
// (point, band) item on the (4M1+1)(4M2+1)(4M3+1) difference grid.
template <int NS>
__global__ void __launch_bounds__(256) sens_correlate(const cd *__restrict__ U, const cd *__restrict__ S, int n_items,
                                                      int d, int M1, int M2, int M3, cd *__restrict__ C) {
  constexpr int NT = NS * (NS + 1) / 2, NF = NT + 1;
  const int n1 = 2 * M1 + 1, n2 = 2 * M2 + 1, n3 = 2 * M3 + 1;
  const int N = n1 * n2 * n3;
  const int q1 = 4 * M1 + 1, q2 = 4 * M2 + 1, q3 = 4 * M3 + 1;
  const int nD = q1 * q2 * q3;
  const int item = blockIdx.y;
  const int D = blockIdx.x * 256 + threadIdx.x;
  if (item >= n_items || D >= nD) return;
  const int dr = D % q3 - 2 * M3, dq = (D / q3) % q2 - 2 * M2, dm = D / q3 / q2 - 2 * M1;
  const cd *u = U + (size_t)item * d * N;
  const cd *sv = S + (size_t)item * NS * N;
  cd acc[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = mk(0.0, 0.0);
  const int a0 = max(0, -dm), a1 = min(n1, n1 - dm);
  const int b0 = max(0, -dq), b1 = min(n2, n2 - dq);
  const int e0 = max(0, -dr), e1 = min(n3, n3 - dr);
  for (int a = a0; a < a1; ++a)
    for (int b = b0; b < b1; ++b)
      for (int e = e0; e < e1; ++e) {
        const int r = (a * n2 + b) * n3 + e;
        const int c = ((a + dm) * n2 + (b + dq)) * n3 + (e + dr);
        cd sr[NS], sc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          sr[s] = gld(sv, (size_t)s * N + r);
          sc[s] = gld(sv, (size_t)s * N + c);
        }
        int f = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int t = s; t < NS; ++t) acc[f] = cfma_cj(sr[s], sc[t], acc[f]), ++f;
        for (int l = 0; l < d; ++l) acc[NT] = cfma_cj(gld(u, (size_t)l * N + r), gld(u, (size_t)l * N + c), acc[NT]);
      }
  cd *out = C + (size_t)item * NF * nD + D;
#pragma unroll
  for (int f = 0; f < NF; ++f) out[(size_t)f * nD] = acc[f];
}

// Adjoint passes over batch b = item * nf + f.
// Y1[b][i][q][r] = sum_m sinc(m/nx) e^{i pi m (2i+1)/nx} C[b][m][q][r]
__global__ void __launch_bounds__(256) sens_pass_x(const cd *__restrict__ C, size_t batches, int nx, int M1, int M2,
                                                   int M3, cd *__restrict__ Y1) {
  const int q1 = 4 * M1 + 1, q2 = 4 * M2 + 1, q3 = 4 * M3 + 1;
  const size_t per = (size_t)nx * q2 * q3;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= batches * per) return;
  const size_t bt = e / per;
  const int qr = (int)(e % ((size_t)q2 * q3));
  const int i = (int)((e / ((size_t)q2 * q3)) % nx);
  const cd *c = C + bt * (size_t)q1 * q2 * q3 + qr;
  cd acc = mk(0.0, 0.0);
  for (int mi = 0; mi < q1; ++mi) {
    const int m = mi - 2 * M1;
    acc = acc + (sincp(m, nx) * c[(size_t)mi * q2 * q3]) * eipi((long)m * (2 * i + 1), nx);
  }
  Y1[e] = acc;
}

// Y2[b][i][j][r] = sum_q sinc(q/ny) e^{i pi q (2j+1)/ny} Y1[b][i][q][r]
__global__ void __launch_bounds__(256) sens_pass_y(const cd *__restrict__ Y1, size_t batches, int nx, int ny, int M2,
                                                   int M3, cd *__restrict__ Y2) {
  const int q2 = 4 * M2 + 1, q3 = 4 * M3 + 1;
  const size_t per = (size_t)nx * ny * q3;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= batches * per) return;
  const int r = (int)(e % q3);
  const int j = (int)((e / q3) % ny);
  const size_t bi = e / q3 / ny;   // b * nx + i
  const cd *y = Y1 + bi * (size_t)q2 * q3 + r;
  cd acc = mk(0.0, 0.0);
  for (int qi = 0; qi < q2; ++qi) {
    const int q = qi - 2 * M2;
    acc = acc + (sincp(q, ny) * y[(size_t)qi * q3]) * eipi((long)q * (2 * j + 1), ny);
  }
  Y2[e] = acc;
}

// G[b][i][j][k] = fac(b) |Omega|/(nx ny nz) Re sum_r sinc(r/nz) e^{i pi r (2k+1)/nz} Y2[b][i][j][r]
// with fac = -1 (s = t), -2 (s < t), -lambda_item (density).
__global__ void __launch_bounds__(256) sens_pass_z(const cd *__restrict__ Y2, int n_items, int nf, int nx, int ny,
                                                   int nz, int M3, double vol, const double *__restrict__ omega,
                                                   int ns, double *__restrict__ G) {
  const int q3 = 4 * M3 + 1;
  const size_t cells = (size_t)nx * ny * nz;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n_items * nf * cells) return;
  const int k = (int)(e % nz);
  const size_t bij = e / nz;              // (b * nx + i) * ny + j
  const size_t bt = e / cells;            // item * nf + f
  const int f = (int)(bt % nf), item = (int)(bt / nf);
  const cd *y = Y2 + bij * q3;
  double acc = 0.0;
  for (int ri = 0; ri < q3; ++ri) {
    const int r = ri - 2 * M3;
    const cd w = eipi((long)r * (2 * k + 1), nz);
    acc += sincp(r, nz) * (y[ri].re * w.re - y[ri].im * w.im);
  }
  double fac;
  if (f == nf - 1) {
    const double om = omega[item];
    fac = -om * om;
  } else {
    // pair index f -> (s, t): off-diagonal pairs move two blocks
    int s = 0, rem = f;
    while (rem >= ns - s) {
      rem -= ns - s;
      ++s;
    }
    fac = rem == 0 ? -1.0 : -2.0;
  }
  G[e] = fac * vol / (double)cells * acc;
}

hipError_t launch_sensitivities(const cd *U, const cd *S, const double *omega, int n_items, int d, int M1, int M2,
                                int M3, int nx, int ny, int nz, double vol, cd *Cw, cd *Y1, cd *Y2, double *G,
                                hipStream_t st) {
  const int ns = d == 2 ? 3 : 6, nf = ns * (ns + 1) / 2 + 1;
  const int nD = (4 * M1 + 1) * (4 * M2 + 1) * (4 * M3 + 1);
  const dim3 gc((nD + 255) / 256, n_items);
  if (d == 2)
    hipLaunchKernelGGL(sens_correlate<3>, gc, dim3(256), 0, st, U, S, n_items, d, M1, M2, M3, Cw);
  else
    hipLaunchKernelGGL(sens_correlate<6>, gc, dim3(256), 0, st, U, S, n_items, d, M1, M2, M3, Cw);
  const size_t B = (size_t)n_items * nf;
  const size_t t1 = B * nx * (4 * M2 + 1) * (4 * M3 + 1), t2 = B * nx * ny * (4 * M3 + 1), t3 = B * nx * ny * nz;
  hipLaunchKernelGGL(sens_pass_x, dim3((unsigned)((t1 + 255) / 256)), dim3(256), 0, st, Cw, B, nx, M1, M2, M3, Y1);
  hipLaunchKernelGGL(sens_pass_y, dim3((unsigned)((t2 + 255) / 256)), dim3(256), 0, st, Y1, B, nx, ny, M2, M3, Y2);
  hipLaunchKernelGGL(sens_pass_z, dim3((unsigned)((t3 + 255) / 256)), dim3(256), 0, st, Y2, n_items, nf, nx, ny, nz,
                     M3, vol, omega, ns, G);
  return hipGetLastError();
}

}  // namespace mvpb
