// Tridiagonal eigenpairs and the FP64 Rayleigh-Ritz refinement of the
// batched Hermitian eigensolve (the reductions live in band.hip).
//  1. Lowest nb eigenvalues of T by multisection on Sturm counts; the
//     eigenvectors of isolated ones by the twisted factorization, those of
//     close clusters by inverse iteration with a pivoted tridiagonal LU and
//     Gram-Schmidt within the cluster.
//  2. FP64 Rayleigh-Ritz on span(Y) with the kept copy of C(k):
//     eigenpairs of Y^H C Y, omega = sqrt(max(lambda, 0)).
#include <float.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {


// ---------------------------------------------------------------------------
// 1. Tridiagonal eigenproblem: multisection for the lowest nb eigenvalues,
//    inverse iteration for the eigenvectors.
// ---------------------------------------------------------------------------
// Reciprocal for the LDL^T pivot recurrences: the hardware reciprocal refined
// by one Newton step (a few ulps per pivot keep them backward stable).
__device__ __forceinline__ double fast_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
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

// Gershgorin bounds of T (every thread receives them); red holds 3 * waves doubles.
MVPB_DEV void gershgorin(const double *dd, const double *ee, int n, double *red, double &gl, double &gu,
                         double &emax2) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  gl = DBL_MAX;
  gu = -DBL_MAX;
  emax2 = 0.0;
  for (int r = tid; r < n; r += blockDim.x) {
    const double er = (r < n - 1) ? ee[r] : 0.0;
    const double el = (r > 0) ? ee[r - 1] : 0.0;
    const double rad = fabs(er) + fabs(el);
    gl = fmin(gl, dd[r] - rad);
    gu = fmax(gu, dd[r] + rad);
    emax2 = fmax(emax2, er * er);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  if (lane == 0) {
    red[3 * wid] = gl;
    red[3 * wid + 1] = gu;
    red[3 * wid + 2] = emax2;
  }
  __syncthreads();
  gl = DBL_MAX;
  gu = -DBL_MAX;
  emax2 = 0.0;
  for (int q = 0; q < nw; ++q) {
    gl = fmin(gl, red[3 * q]);
    gu = fmax(gu, red[3 * q + 1]);
    emax2 = fmax(emax2, red[3 * q + 2]);
  }
  __syncthreads();
}

// Number of eigenvalues of T below x without divisions: the signs of the
// leading principal minors p_k = det(T_k - x I), from the three-term
// recurrence p_{k+1} = (d_k - x) p_k - e_{k-1}^2 p_{k-1} (a Sturm sequence:
// every change of sign between consecutive minors is one eigenvalue below
// x).  Each step is one dependent FMA.  Every 8 steps both carried minors are
// multiplied by the same power of two, which keeps the signs exactly; with
// T scaled to |T| = O(1) a minor changes by at most 3^8 between rescalings.
// A minor that is exactly zero counts as positive: the next minor,
// -e^2 p_{k-1}, then supplies the one change of sign the zero stands for.
// e2p[k] = e_{k-1}^2 (e2p[0] = 0).
constexpr int SC_CHUNK = 8;
__device__ __forceinline__ int sturm_count_minors(const double *__restrict__ dd, const double *__restrict__ e2p,
                                                  int n, double x) {
  double pp = 0.0, p = 1.0;
  int cnt = 0, k = 0;
  for (; k + SC_CHUNK <= n; k += SC_CHUNK) {
    double dc[SC_CHUNK], ec[SC_CHUNK];
#pragma unroll
    for (int u = 0; u < SC_CHUNK; ++u) {
      dc[u] = dd[k + u] - x;
      ec[u] = e2p[k + u];
    }
#pragma unroll
    for (int u = 0; u < SC_CHUNK; ++u) {
      const double pn = fma(dc[u], p, -ec[u] * pp);
      cnt += (pn < 0.0) != (p < 0.0);
      pp = p;
      p = pn;
    }
    int ex = 0;
    (void)frexp(p, &ex);
    p = ldexp(p, -ex);
    pp = ldexp(pp, -ex);
  }
  for (; k < n; ++k) {
    const double pn = fma(dd[k] - x, p, -e2p[k] * pp);
    cnt += (pn < 0.0) != (p < 0.0);
    pp = p;
    p = pn;
  }
  return cnt;
}

// 1a. The lowest nb eigenvalues of T by multisection.  BISI_GROUPS
// workgroups per item, workgroup g bracketing eigenvalues g, g + BISI_GROUPS,
// ...  The first round spreads BISI_THREADS probes over the Gershgorin
// interval, and every eigenvalue takes its bracket from their counts; later
// rounds deal the probes out evenly over the eigenvalues whose bracket is
// still wider than a few ulps of |T|.
constexpr int BISI_THREADS = 256;
constexpr int BISI_GROUPS = 4;
constexpr int BISI_MAX = MAX_BANDS / BISI_GROUPS;   // eigenvalues of one workgroup
static_assert(BISI_MAX * BISI_GROUPS == MAX_BANDS && BISI_MAX <= BISI_THREADS / 4, "probes per open eigenvalue");
__global__ void __launch_bounds__(BISI_THREADS) tridiag_bisect_item(const EigItem *__restrict__ items) {
  extern __shared__ double shd[];   // dd (n), ee (n), e2p (n + 1)
  __shared__ double red[3 * (BISI_THREADS / 64)];
  __shared__ double xs[BISI_THREADS];
  __shared__ int cnt_s[BISI_THREADS];
  __shared__ int first_s[BISI_THREADS / 64][BISI_MAX];
  __shared__ double lo_s[BISI_MAX], hi_s[BISI_MAX];
  __shared__ int act_s[BISI_MAX];
  __shared__ int nact_s;
  const EigItem it = items[blockIdx.y];
  const int n = it.n, nb_all = it.nb, g0 = blockIdx.x;
  if (g0 >= nb_all) return;
  const int nb = (nb_all - g0 + BISI_GROUPS - 1) / BISI_GROUPS;   // eigenvalues of this workgroup
  double *dd = shd, *ee = dd + n, *e2p = ee + n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int r = tid; r < n; r += BISI_THREADS) {
    dd[r] = it.d[r];
    ee[r] = (r < n - 1) ? it.e[r] : 0.0;
  }
  __syncthreads();
  double gl, gu, emax2;
  gershgorin(dd, ee, n, red, gl, gu, emax2);
  const double bnorm = fmax(fabs(gl), fabs(gu));
  // exact power-of-two scale that brings |T| near 1
  int sex = 0;
  if (bnorm > 0.0) (void)frexp(bnorm, &sex);
  for (int r = tid; r < n; r += BISI_THREADS) {
    dd[r] = ldexp(dd[r], -sex);
    const double er = ldexp(r > 0 ? ee[r - 1] : 0.0, -sex);
    e2p[r] = er * er;
  }
  const double bn = ldexp(bnorm, -sex);
  const double slack = 2.0 * DBL_EPSILON * bn * n;
  const double glo = ldexp(gl, -sex) - slack, ghi = ldexp(gu, -sex) + slack;
  const double tol_abs = 2.0 * DBL_EPSILON * bn;
  __syncthreads();
  // pass 0: one set of probes for every eigenvalue
  {
    const double x = glo + (ghi - glo) * (double)(tid + 1) / (double)(BISI_THREADS + 1);
    xs[tid] = x;
    const int c = sturm_count_minors(dd, e2p, n, x);
    for (int j = 0; j < nb; ++j) {
      const unsigned long long bal = __ballot(c > g0 + BISI_GROUPS * j);
      if (lane == 0) first_s[w][j] = bal ? w * 64 + __builtin_ctzll(bal) : BISI_THREADS;
    }
    __syncthreads();
    if (tid < nb) {
      int g = BISI_THREADS;
      for (int q = 0; q < BISI_THREADS / 64; ++q) g = min(g, first_s[q][tid]);
      lo_s[tid] = (g > 0) ? xs[g - 1] : glo;
      hi_s[tid] = (g < BISI_THREADS) ? xs[g] : ghi;
    }
    __syncthreads();
  }
  for (int round = 0; round < 24; ++round) {
    if (tid == 0) {
      int na = 0;
      for (int j = 0; j < nb; ++j) {
        const double lo = lo_s[j], hi = hi_s[j];
        if (hi - lo > fmax(tol_abs, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) act_s[na++] = j;
      }
      nact_s = na;
    }
    __syncthreads();
    const int na = nact_s;
    if (na == 0) break;
    const int P = BISI_THREADS / na;   // probes per open eigenvalue (>= 4 for nb <= MAX_BANDS)
    const int a = tid / P, pq = tid % P;
    if (a < na) {
      const int j = act_s[a];
      const double lo = lo_s[j], hi = hi_s[j];
      const double x = lo + (hi - lo) * (double)(pq + 1) / (double)(P + 1);
      xs[tid] = x;
      cnt_s[tid] = sturm_count_minors(dd, e2p, n, x);
    }
    __syncthreads();
    if (tid < na) {
      const int j = act_s[tid];
      const int jg = g0 + BISI_GROUPS * j;   // index among all eigenvalues
      int g = P;
      for (int q = 0; q < P; ++q)
        if (cnt_s[tid * P + q] > jg) {
          g = q;
          break;
        }
      const double lo = lo_s[j], hi = hi_s[j];
      lo_s[j] = (g > 0) ? xs[tid * P + g - 1] : lo;
      hi_s[j] = (g < P) ? xs[tid * P + g] : hi;
    }
    __syncthreads();
  }
  if (tid < nb) it.lam_t[g0 + BISI_GROUPS * tid] = ldexp(0.5 * (lo_s[tid] + hi_s[tid]), sex);
}

// Sequential kernels of inverse iteration (one lane).  The recurrences run in
// chunks of 8 steps whose operands are loaded one chunk ahead, so that LDS
// latency is paid once per chunk and overlaps the arithmetic.
constexpr int TCH = 8;

// One pivoted elimination step of T - sh I (row r): state (dr, ur) in, out.
MVPB_DEV void lu_step(int r, double lr, double dns, double un, double pert, double &dr, double &ur,
                      double *__restrict__ DL, double *__restrict__ DGi, double *__restrict__ DU,
                      double *__restrict__ DU2, double *__restrict__ PV, double &fo, bool &sw) {
  // pivot row: the current one if |dr| >= |lr|, else the next (swap); the
  // two cases by selects, so that the dependent chain has no branch
  const bool keep = fabs(dr) >= fabs(lr);
  const double piv = keep ? dr : lr;   // lr != 0 when it is the pivot
  const double ip = fast_rcp(piv == 0.0 ? pert : piv);
  const double f = (keep ? lr : dr) * ip;
  DGi[r] = ip;
  DU[r] = keep ? ur : dns;
  DU2[r] = keep ? 0.0 : un;
  DL[r] = f;
  PV[r] = keep ? 0.0 : 1.0;
  dr = (keep ? dns : ur) - f * (keep ? ur : dns);
  ur = keep ? un : -f * un;
  fo = f;
  sw = !keep;
}

// Forward step r of (P, L)^-1 applied to x: with the carried value cur (row r
// after the earlier steps) and x[r+1], writes x[r] and carries row r+1.
MVPB_DEV void fwd_step(int r, bool sw, double f, double nxt, double &cur, double *__restrict__ xv) {
  const double br = sw ? nxt : cur;
  const double br1 = sw ? cur : nxt;
  xv[r] = br;
  cur = br1 - f * br;
}

// LU with partial pivoting of T - sh I: multipliers DL, reciprocal pivots DGi,
// first and second superdiagonal of U (DU, DU2), row swaps PV (0/1).  With
// FWD, the forward substitution of x <- (T - sh I)^-1 x runs in the same pass
// (the same operations as in tri_solve, one row behind the factorisation).
template <bool FWD>
MVPB_DEV void tri_lu(const double *__restrict__ dd, const double *__restrict__ ee, int n, double sh, double pert,
                     double *__restrict__ DL, double *__restrict__ DGi, double *__restrict__ DU,
                     double *__restrict__ DU2, double *__restrict__ PV, double *__restrict__ xv) {
  double dr = dd[0] - sh, ur = (n > 1) ? ee[0] : 0.0;
  double cur = FWD ? xv[0] : 0.0;
  double f;
  bool sw;
  int r = 0;
  // a full chunk at r needs ee[r .. r+TCH], dd[r+1 .. r+TCH] and xv[r+1 .. r+TCH], all < n-1 / < n
  if (r + TCH < n - 1) {
    double ec[TCH + 1], dc[TCH], xc[TCH];
#pragma unroll
    for (int u = 0; u <= TCH; ++u) ec[u] = ee[r + u];
#pragma unroll
    for (int u = 0; u < TCH; ++u) {
      dc[u] = dd[r + 1 + u];
      xc[u] = FWD ? xv[r + 1 + u] : 0.0;
    }
    for (; r + TCH < n - 1; r += TCH) {
      double en[TCH + 1], dn[TCH], xn[TCH];
      const bool more = r + 2 * TCH < n - 1;
      if (more) {
#pragma unroll
        for (int u = 0; u <= TCH; ++u) en[u] = ee[r + TCH + u];
#pragma unroll
        for (int u = 0; u < TCH; ++u) {
          dn[u] = dd[r + TCH + 1 + u];
          xn[u] = FWD ? xv[r + TCH + 1 + u] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < TCH; ++u) {
        lu_step(r + u, ec[u], dc[u] - sh, ec[u + 1], pert, dr, ur, DL, DGi, DU, DU2, PV, f, sw);
        if (FWD) fwd_step(r + u, sw, f, xc[u], cur, xv);
      }
      if (more) {
#pragma unroll
        for (int u = 0; u <= TCH; ++u) ec[u] = en[u];
#pragma unroll
        for (int u = 0; u < TCH; ++u) {
          dc[u] = dn[u];
          xc[u] = xn[u];
        }
      }
    }
  }
  for (; r < n - 1; ++r) {
    lu_step(r, ee[r], dd[r + 1] - sh, (r < n - 2) ? ee[r + 1] : 0.0, pert, dr, ur, DL, DGi, DU, DU2, PV, f, sw);
    if (FWD) fwd_step(r, sw, f, xv[r + 1], cur, xv);
  }
  DGi[n - 1] = fast_rcp(dr == 0.0 ? pert : dr);
  if (FWD) xv[n - 1] = cur;
}

// Forward part of tri_solve: apply P and L^-1.  Step r reads x[r+1], PV[r],
// DL[r]; writes x[r].
MVPB_DEV void tri_solve_fwd(double *__restrict__ xv, int n, const double *__restrict__ DL,
                            const double *__restrict__ PV) {
  double cur = xv[0];
  int r = 0;
  if (r + TCH < n - 1) {
    double xc[TCH], pc[TCH], lc[TCH];
#pragma unroll
    for (int u = 0; u < TCH; ++u) {
      xc[u] = xv[r + 1 + u];
      pc[u] = PV[r + u];
      lc[u] = DL[r + u];
    }
    for (; r + TCH < n - 1; r += TCH) {
      double xn[TCH], pn[TCH], ln[TCH];
      const bool more = r + 2 * TCH < n - 1;
      if (more) {
#pragma unroll
        for (int u = 0; u < TCH; ++u) {
          xn[u] = xv[r + TCH + 1 + u];
          pn[u] = PV[r + TCH + u];
          ln[u] = DL[r + TCH + u];
        }
      }
#pragma unroll
      for (int u = 0; u < TCH; ++u) {
        const bool sw = pc[u] != 0.0;
        const double br = sw ? xc[u] : cur;
        const double br1 = sw ? cur : xc[u];
        xv[r + u] = br;
        cur = br1 - lc[u] * br;
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < TCH; ++u) {
          xc[u] = xn[u];
          pc[u] = pn[u];
          lc[u] = ln[u];
        }
      }
    }
  }
  for (; r < n - 1; ++r) {
    const double nxt = xv[r + 1];
    const bool sw = PV[r] != 0.0;
    const double br = sw ? nxt : cur;
    const double br1 = sw ? cur : nxt;
    xv[r] = br;
    cur = br1 - DL[r] * br;
  }
  xv[n - 1] = cur;
}

// Backward part of tri_solve: substitution with U.
MVPB_DEV void tri_solve_back(double *__restrict__ xv, int n, const double *__restrict__ DGi,
                             const double *__restrict__ DU, const double *__restrict__ DU2) {
  // backward substitution with U, rows n-1 .. 0.  Step r reads x[r], DU[r],
  // DU2[r], DGi[r]; writes x[r].  Rescaling (rare) touches the rows above r.
  double x1 = 0.0, x2 = 0.0, sc = 1.0;
  // C1, C2: the terms of rows q+1, q+2 exist (every row but the last two)
  auto bstep = [&](auto c1, auto c2, int q, double b, double u1, double u2, double gi) {
    double sacc = sc * b;
    if (decltype(c1)::value) sacc -= u1 * x1;
    if (decltype(c2)::value) sacc -= u2 * x2;
    double x = sacc * gi;
    if (!(fabs(x) <= 1e150)) {   // not finite, or too large: one test on the common path
      if (!isfinite(x)) {
        x = 0.0;
      } else {
        // keep the iterate finite: rescale what is solved and what is left
        const double f = 1e-150;
        for (int t = q + 1; t < n; ++t) xv[t] *= f;
        x1 *= f;
        x2 *= f;
        sc *= f;
        x *= f;
      }
    }
    xv[q] = x;
    x2 = x1;
    x1 = x;
  };
  using T0 = std::integral_constant<bool, false>;
  using T1 = std::integral_constant<bool, true>;
  int rr = n - 1;
  if (rr >= 0) bstep(T0{}, T0{}, rr, xv[rr], DU[rr], DU2[rr], DGi[rr]);
  --rr;
  if (rr >= 0) bstep(T1{}, T0{}, rr, xv[rr], DU[rr], DU2[rr], DGi[rr]);
  --rr;
  if (rr - TCH + 1 >= 0) {
    double bc[TCH], uc[TCH], vc[TCH], gc[TCH];
#pragma unroll
    for (int u = 0; u < TCH; ++u) {
      const int q = rr - u;
      bc[u] = xv[q];
      uc[u] = DU[q];
      vc[u] = DU2[q];
      gc[u] = DGi[q];
    }
    for (; rr - TCH + 1 >= 0; rr -= TCH) {
      double bn[TCH], un[TCH], vn[TCH], gn[TCH];
      const bool more = rr - 2 * TCH + 1 >= 0;
      if (more) {
#pragma unroll
        for (int u = 0; u < TCH; ++u) {
          const int q = rr - TCH - u;
          bn[u] = xv[q];
          un[u] = DU[q];
          vn[u] = DU2[q];
          gn[u] = DGi[q];
        }
      }
#pragma unroll
      for (int u = 0; u < TCH; ++u) bstep(T1{}, T1{}, rr - u, bc[u], uc[u], vc[u], gc[u]);
      if (more) {
#pragma unroll
        for (int u = 0; u < TCH; ++u) {
          bc[u] = bn[u];
          uc[u] = un[u];
          vc[u] = vn[u];
          gc[u] = gn[u];
        }
      }
    }
  }
  for (; rr >= 0; --rr) bstep(T1{}, T1{}, rr, xv[rr], DU[rr], DU2[rr], DGi[rr]);
}

// x <- (T - sh I)^-1 x with the factors of tri_lu (x in place); fwd = false
// when tri_lu has already applied the forward part.
MVPB_DEV void tri_solve(double *__restrict__ xv, int n, const double *__restrict__ DL,
                        const double *__restrict__ DGi, const double *__restrict__ DU,
                        const double *__restrict__ DU2, const double *__restrict__ PV, bool fwd = true) {
  if (fwd) tri_solve_fwd(xv, n, DL, PV);
  tri_solve_back(xv, n, DGi, DU, DU2);
}

// Eigenvalues closer than CLUSTER_REL |T| to a neighbour form a cluster: their
// eigenvectors come from inverse iteration with Gram-Schmidt (1b); isolated
// ones from the twisted factorization (1c).
constexpr double CLUSTER_REL = 1e-9;
MVPB_DEV bool in_cluster(const double *lam, int j, int nb, double thr) {
  return (j > 0 && lam[j] - lam[j - 1] <= thr) || (j + 1 < nb && lam[j + 1] - lam[j] <= thr);
}

// 1c. Eigenvector of an isolated eigenvalue lam by the twisted factorization
// of T - lam I: the pivots of the top-down (dp) and bottom-up (dm) LDL^T
// factorizations, computed side by side by two lanes; the twist index r
// minimising |gamma_r| = |dp_r + dm_r - (d_r - lam)|; then z_r = 1 and
// z_i = -(e_i / dp_i) z_{i+1} above r, z_i = -(e_{i-1} / dm_i) z_{i-1} below,
// again on two lanes (the ratios are formed by the whole wavefront first).
// Isolated means a gap above CLUSTER_REL |T| to both neighbours: the vector's
// residual is of order sqrt(n) eps |T|, and the Rayleigh-Ritz step that
// follows turns it into an eigenvalue error of order residual^2 / gap.  One
// wavefront per eigenvalue; lane 0 runs the top-down and lane 1 the bottom-up
// recurrences in one instruction stream (no divergent branches), their
// operands loaded a chunk ahead.
__global__ void __launch_bounds__(64) tridiag_twisted(const EigItem *__restrict__ items) {
  extern __shared__ double shd[];   // dd, ee, dp, dm (n each)
  __shared__ double red[3];
  const EigItem it = items[blockIdx.y];
  const int n = it.n, nb = it.nb, j = blockIdx.x;
  if (j >= nb) return;
  const int lane = threadIdx.x;
  double *dd = shd, *ee = dd + n, *dp = ee + n, *dm = dp + n;
  for (int r = lane; r < n; r += 64) {
    dd[r] = it.d[r];
    ee[r] = (r < n - 1) ? it.e[r] : 0.0;
  }
  __syncthreads();
  double gl, gu, emax2;
  gershgorin(dd, ee, n, red, gl, gu, emax2);
  const double bnorm = fmax(fabs(gl), fabs(gu));
  const double thr = CLUSTER_REL * bnorm;
  const double *lam = it.lam_t;
  const double lj = lam[j];
  if (in_cluster(lam, j, nb, thr)) return;   // cluster member: inverse iteration
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  // lane 0: dp_i = (d_i - lam) - e_{i-1}^2 / dp_{i-1}, i = 0 .. n-1;
  // lane 1: dm_i = (d_i - lam) - e_i^2 / dm_{i+1}, i = n-1 .. 0
  if (lane < 2) {
    const bool fw = lane == 0;
    double *dst = fw ? dp : dm;
    const int step = fw ? 1 : -1;
    int i = fw ? 0 : n - 1;
    // e index of step t: fw: i - 1, bw: i (zero where absent)
    double q = dd[i] - lj;
    if (fabs(q) < pivmin) q = -pivmin;
    dst[i] = q;
    int t = 1;
    constexpr int CH = 8;
    for (; t + CH <= n; t += CH) {
      double dc[CH], ec[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int ii = i + step * (u + 1);
        dc[u] = dd[ii] - lj;
        const double e = ee[fw ? ii - 1 : ii];
        ec[u] = e * e;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        q = dc[u] - ec[u] * fast_rcp(q);
        if (fabs(q) < pivmin) q = -pivmin;
        dst[i + step * (u + 1)] = q;
      }
      i += step * CH;
    }
    for (; t < n; ++t) {
      i += step;
      const double e = ee[fw ? i - 1 : i];
      q = (dd[i] - lj) - e * e * fast_rcp(q);
      if (fabs(q) < pivmin) q = -pivmin;
      dst[i] = q;
    }
  }
  __syncthreads();
  // twist index: smallest |gamma|, lowest index on ties
  double gbest = DBL_MAX;
  int rbest = 0;
  for (int i = lane; i < n; i += 64) {
    const double g = fabs(dp[i] + dm[i] - (dd[i] - lj));
    if (g < gbest) {
      gbest = g;
      rbest = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double go = __shfl_xor(gbest, o, 64);
    const int ro = __shfl_xor(rbest, o, 64);
    if (go < gbest || (go == gbest && ro < rbest)) {
      gbest = go;
      rbest = ro;
    }
  }
  const int r = rbest;
  // ratios in place: dp[i] <- -e_i / dp_i (i < r), dm[i] <- -e_{i-1} / dm_i (i > r)
  for (int i = lane; i < n; i += 64) {
    if (i < r) dp[i] = -ee[i] / dp[i];
    if (i > r) dm[i] = -ee[i - 1] / dm[i];
  }
  __syncthreads();
  // z above r (lane 0, in dp) and below r (lane 1, in dm): products of the ratios
  if (lane < 2) {
    const bool up = lane == 0;
    double *buf = up ? dp : dm;
    const int step = up ? -1 : 1;
    const int len = up ? r : n - 1 - r;
    double z = 1.0;
    int i = r;
    for (int t = 0; t < len; ++t) {
      i += step;
      z *= buf[i];
      buf[i] = z;
    }
  }
  __syncthreads();
  double s2 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double z = i < r ? dp[i] : (i > r ? dm[i] : 1.0);
    s2 = fma(z, z, s2);
  }
  s2 = wave_sum(s2);
  const double inv = 1.0 / sqrt(s2);
  double *X = it.X;
  for (int i = lane; i < n; i += 64) {
    const double z = i < r ? dp[i] : (i > r ? dm[i] : 1.0);
    gst(X, (size_t)i * nb + j, z * inv);
  }
}

// 1b. Eigenvectors of cluster members (eigenvalues within CLUSTER_REL |T|
// of a neighbour) by inverse iteration with a pivoted LU of T - lam I: one
// solve from a pseudo-random start that differs per member, so that members
// of a (near-)degenerate cluster come out independent.  With the shift within
// about eps |T| of the eigenvalue, one solve leaves the components outside
// the cluster smaller by the ratio of that distance to the gap; the
// Gram-Schmidt pass below and the Rayleigh-Ritz step after the
// back-transform act on what remains.  One wavefront per
// member, all members at once; lane 0 runs the sequential factorisation and
// solves, the wavefront the normalisation.  tridiag_cluster_gs then
// orthonormalises every cluster.  LU_LDS: the five LU arrays live in LDS
// (else in the item's global scratch).
constexpr int INV_LDS_MAX_N = 2400;
constexpr int INVIT_SOLVES = 1;
template <bool LU_LDS>
__global__ void __launch_bounds__(64) tridiag_invit(const EigItem *__restrict__ items) {
  extern __shared__ double shd[];
  __shared__ double red[3];
  const EigItem it = items[blockIdx.y];
  const int n = it.n, nb = it.nb, jm = blockIdx.x;
  if (jm >= nb) return;
  const int lane = threadIdx.x;
  double *dd = shd, *ee = dd + n, *xv = ee + n;
  double *lub = LU_LDS ? xv + n : it.lu + (size_t)5 * n * jm;
  double *DL = lub, *DGi = lub + n, *DU = lub + 2 * n, *DU2 = lub + 3 * n, *PV = lub + 4 * n;
  for (int r = lane; r < n; r += 64) {
    dd[r] = it.d[r];
    ee[r] = (r < n - 1) ? it.e[r] : 0.0;
  }
  __syncthreads();
  double gl, gu, emax2;
  gershgorin(dd, ee, n, red, gl, gu, emax2);
  const double bnorm = fmax(fabs(gl), fabs(gu));
  const double *lam = it.lam_t;
  if (!in_cluster(lam, jm, nb, CLUSTER_REL * bnorm)) return;   // isolated: twisted factorization
  const double pert = fmax(DBL_EPSILON * bnorm, 1e-280);
  const double sh = lam[jm];
  for (int r = lane; r < n; r += 64) xv[r] = hash_uniform(r + 1, jm + 7);
  __syncthreads();
  // the factorisation carries the forward part of the first solve
  if (lane == 0) tri_lu<true>(dd, ee, n, sh, pert, DL, DGi, DU, DU2, PV, xv);
  for (int iter = 0; iter < INVIT_SOLVES; ++iter) {
    if (lane == 0) tri_solve(xv, n, DL, DGi, DU, DU2, PV, iter > 0);
    __syncthreads();
    double amax = 0.0;
    for (int r = lane; r < n; r += 64) amax = fmax(amax, fabs(xv[r]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    const double ia = amax > 0.0 ? 1.0 / amax : 1.0;
    double s2 = 0.0;
    for (int r = lane; r < n; r += 64) {
      const double v = xv[r] * ia;
      s2 = fma(v, v, s2);
    }
    s2 = wave_sum(s2);
    const double inv = s2 > 0.0 ? ia / sqrt(s2) : 0.0;
    for (int r = lane; r < n; r += 64) xv[r] *= inv;
    __syncthreads();
  }
  double *X = it.X;
  for (int r = lane; r < n; r += 64) gst(X, (size_t)r * nb + jm, xv[r]);
}

// 1b'. Modified Gram-Schmidt (two passes) over the eigenvectors of every
// cluster, in eigenvalue order; one wavefront per cluster, started by the
// wavefront of the cluster's first member.
__global__ void __launch_bounds__(64) tridiag_cluster_gs(const EigItem *__restrict__ items) {
  __shared__ double red[3];
  const EigItem it = items[blockIdx.y];
  const int n = it.n, nb = it.nb, j0 = blockIdx.x;
  if (j0 >= nb) return;
  const int lane = threadIdx.x;
  // |T| from the Gershgorin bounds, read straight from d and e
  double gl = DBL_MAX, gu = -DBL_MAX;
  for (int r = lane; r < n; r += 64) {
    const double er = (r < n - 1) ? fabs(it.e[r]) : 0.0, el = (r > 0) ? fabs(it.e[r - 1]) : 0.0;
    gl = fmin(gl, it.d[r] - er - el);
    gu = fmax(gu, it.d[r] + er + el);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
  }
  (void)red;
  const double thr = CLUSTER_REL * fmax(fabs(gl), fabs(gu));
  const double *lam = it.lam_t;
  if (j0 > 0 && lam[j0] - lam[j0 - 1] <= thr) return;   // not the first member
  int j1 = j0 + 1;
  while (j1 < nb && lam[j1] - lam[j1 - 1] <= thr) ++j1;
  if (j1 == j0 + 1) return;                              // isolated
  double *X = it.X;
  for (int jm = j0; jm < j1; ++jm) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = j0; q < jm; ++q) {
        double dot = 0.0;
        for (int r = lane; r < n; r += 64) dot = fma(gld(X, (size_t)r * nb + q), gld(X, (size_t)r * nb + jm), dot);
        dot = wave_sum(dot);
        for (int r = lane; r < n; r += 64)
          gst(X, (size_t)r * nb + jm, fma(-dot, gld(X, (size_t)r * nb + q), gld(X, (size_t)r * nb + jm)));
      }
      double s2 = 0.0;
      for (int r = lane; r < n; r += 64) {
        const double v = gld(X, (size_t)r * nb + jm);
        s2 = fma(v, v, s2);
      }
      s2 = wave_sum(s2);
      const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
      for (int r = lane; r < n; r += 64) gst(X, (size_t)r * nb + jm, gld(X, (size_t)r * nb + jm) * inv);
    }
  }
}

hipError_t launch_tridiag_eig(const EigItem *items, int n_items, int n_max, int nb, hipStream_t st,
                              hipStream_t side, hipEvent_t ev_fork, hipEvent_t ev_join) {
  ProfScope ps(K_TRIDIAG, st);
  hipLaunchKernelGGL(tridiag_bisect_item, dim3(BISI_GROUPS, n_items), dim3(BISI_THREADS),
                     sizeof(double) * (3 * n_max + 1), st, items);
  const bool two = side != nullptr && ev_fork != nullptr && ev_join != nullptr;
  hipStream_t si = st;
  if (two) {
    hipError_t e = hipEventRecord(ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, ev_fork, 0);
    if (e != hipSuccess) return e;
    si = side;
  }
  if (n_max <= INV_LDS_MAX_N)
    hipLaunchKernelGGL(tridiag_invit<true>, dim3(nb, n_items), dim3(64), sizeof(double) * 8 * n_max, si, items);
  else
    hipLaunchKernelGGL(tridiag_invit<false>, dim3(nb, n_items), dim3(64), sizeof(double) * 3 * n_max, si, items);
  hipLaunchKernelGGL(tridiag_twisted, dim3(nb, n_items), dim3(64), sizeof(double) * 4 * n_max, st, items);
  if (two) {
    hipError_t e = hipEventRecord(ev_join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev_join, 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(tridiag_cluster_gs, dim3(nb, n_items), dim3(64), 0, st, items);
  return hipGetLastError();
}

// Cyclic Jacobi on the Hermitian nb x nb matrix G (LDS), rotations
// accumulated into V; parallel round-robin pairing over nbe (even) indices.
MVPB_DEV void jacobi_eig(cd (*Gs)[RR_MAX_BANDS + 1], cd (*Vs)[RR_MAX_BANDS + 1], int nb, double *rc, double *rs,
                         cd *rph, int *pa, int *pb) {
  const int tid = threadIdx.x, T = blockDim.x;
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
      for (int e = tid; e < npair * nb; e += T) {
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
      for (int e = tid; e < npair * nb; e += T) {
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
}

// ---------------------------------------------------------------------------
// 2. Rayleigh-Ritz in FP64 on span(Y), Y = the back-transformed eigenvectors
//    (orthonormal up to the inverse iteration's accuracy):
//    rr_product  Z = C Y over 64-row blocks of the kept copy of C(k), and the
//                blocks' Gram partials Y_b^H Z_b, Y_b^H Y_b;
//    rr_small    G = Y^H C Y, M = Y^H Y; M = L L^H; eigenpairs of
//                L^-1 G L^-H (cyclic Jacobi, parallel round-robin pairs);
//                vectors Y L^-H V, lambda ascending, omega = sqrt(max(lambda, 0));
//                items with an error estimate (FP32 reduction) also get the
//                residuals of the refined pairs, a second rr_product pass over
//                them and rr_estimate.
// ---------------------------------------------------------------------------
constexpr int RR_MAXB = RR_MAX_BANDS;
constexpr int RRP_BC_MAX = 24;   // bands per pass of the product kernel (at most)

// RES: the residual pass of items with an error estimate (the vectors are the
// residuals R that rr_small left in the inverse-iteration scratch; only the
// Gram partials R^H C R, R^H R are kept).
template <bool RES, int RRP_BC>
__global__ void __launch_bounds__(256) rr_product(const EigItem *__restrict__ items) {
  extern __shared__ __align__(16) unsigned char rr_raw[];
  __shared__ cd Ys[64][RRP_BC + 1];
  const EigItem it = items[blockIdx.y];
  if (RES && !it.check) return;
  const int n = it.n, nb = it.nb;
  const int rb = blockIdx.x, r0 = rb * 64;
  if (r0 >= n) return;
  const size_t ld = (size_t)n;
  cd *Yr = (cd *)rr_raw;       // [64][nb]
  cd *Zr = Yr + 64 * nb;       // [64][nb]
  const int tid = threadIdx.x, r = tid & 63, ks = tid >> 6;
  const cd *__restrict__ Y = RES ? (const cd *)it.lu : it.Y;
  const cd *__restrict__ Cm = it.Ak;
  const int rows = min(64, n - r0);
  for (int e = tid; e < 64 * nb; e += 256) {
    const int rr = e % 64, b = e / 64;
    Yr[rr * nb + b] = (rr < rows) ? gld(Y, (size_t)b * ld + r0 + rr) : mk(0.0, 0.0);
  }
  for (int b0 = 0; b0 < nb; b0 += RRP_BC) {
    const int bc = min(RRP_BC, nb - b0);
    cd acc[RRP_BC];
#pragma unroll
    for (int b = 0; b < RRP_BC; ++b) acc[b] = mk(0.0, 0.0);
    for (int c0 = 0; c0 < n; c0 += 64) {
      // a full block's 16 entries of C for this thread are loaded at once,
      // before the Y block is staged (same summation order as the loop below)
      const int cmax = min(64, n - c0);
      const bool full = cmax == 64 && r < rows;
      cd a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] = gld(Cm, full ? (size_t)(c0 + ks + 4 * u) * ld + r0 + r : 0);
      __syncthreads();
      for (int e = tid; e < 64 * RRP_BC; e += 256) {
        const int cc = e % 64, b = e / 64;
        Ys[cc][b] = (c0 + cc < n && b < bc) ? gld(Y, (size_t)(b0 + b) * ld + c0 + cc) : mk(0.0, 0.0);
      }
      __syncthreads();
      if (full) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
          for (int b = 0; b < RRP_BC; ++b) acc[b] = cfma(a[u], Ys[ks + 4 * u][b], acc[b]);
      } else if (r < rows) {
        for (int cc = ks; cc < cmax; cc += 4) {
          const cd av = gld(Cm, (size_t)(c0 + cc) * ld + r0 + r);
#pragma unroll
          for (int b = 0; b < RRP_BC; ++b) acc[b] = cfma(av, Ys[cc][b], acc[b]);
        }
      }
    }
    // sum the four column phases into Zr
    for (int ph = 0; ph < 4; ++ph) {
      if (ks == ph) {
#pragma unroll
        for (int b = 0; b < RRP_BC; ++b)
          if (b < bc) Zr[r * nb + b0 + b] = (ph == 0) ? acc[b] : Zr[r * nb + b0 + b] + acc[b];
      }
      __syncthreads();
    }
  }
  cd *Z = it.Z;
  if (!RES)
    for (int e = tid; e < rows * nb; e += 256) {
      const int rr = e % rows, b = e / rows;
      gst(Z, (size_t)b * ld + r0 + rr, Zr[rr * nb + b]);
    }
  // Gram partials of this row block: [0] Y^H Z, [1] Y^H Y
  cd *Gp = it.Gp + (size_t)rb * 2 * nb * nb;
  for (int e = tid; e < nb * nb; e += 256) {
    const int a = e % nb, b = e / nb;
    cd g = mk(0.0, 0.0), m = mk(0.0, 0.0);
    for (int rr = 0; rr < rows; ++rr) {
      const cd ya = Yr[rr * nb + a];
      g = cfma_cj(ya, Zr[rr * nb + b], g);
      m = cfma_cj(ya, Yr[rr * nb + b], m);
    }
    gst(Gp, e, g);
    gst(Gp, (size_t)nb * nb + e, m);
  }
}

__global__ void __launch_bounds__(256) rr_small(const EigItem *__restrict__ items) {
  constexpr int T = 256;
  __shared__ cd Gs[RR_MAXB][RR_MAXB + 1];
  __shared__ cd Vs[RR_MAXB][RR_MAXB + 1];
  __shared__ double rc[RR_MAXB / 2 + 1], rs[RR_MAXB / 2 + 1];
  __shared__ cd rph[RR_MAXB / 2 + 1];
  __shared__ int pa[RR_MAXB / 2 + 1], pb[RR_MAXB / 2 + 1];
  __shared__ int perm[RR_MAXB];
  __shared__ double evs[RR_MAXB];
  const EigItem it = items[blockIdx.x];
  const int n = it.n, nb = it.nb;
  const int tid = threadIdx.x;
  const size_t ld = (size_t)n;
  const int nrb = (n + 63) / 64;
  // G (Hermitian part) and M from the row-block partials
  for (int e = tid; e < nb * nb; e += T) {
    const int a = e % nb, b = e / nb;
    cd g = mk(0.0, 0.0), m = mk(0.0, 0.0);
    for (int q = 0; q < nrb; ++q) {
      const cd *P = it.Gp + (size_t)q * 2 * nb * nb;
      g = g + gld(P, e);
      m = m + gld(P, (size_t)nb * nb + e);
    }
    Gs[a][b] = g;
    Vs[a][b] = m;
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += T) {
    const int a = e % nb, b = e / nb;
    if (a < b) {
      const cd x = Gs[a][b], y2 = Gs[b][a];
      const cd hm = mk(0.5 * (x.re + y2.re), 0.5 * (x.im - y2.im));
      Gs[a][b] = hm;
      Gs[b][a] = conj(hm);
    } else if (a == b) {
      Gs[a][a].im = 0.0;
      Vs[a][a].im = 0.0;
    }
  }
  __syncthreads();
  // Cholesky M = L L^H in Vs (lower), column by column
  for (int j = 0; j < nb; ++j) {
    const double piv = sqrt(fmax(Vs[j][j].re, 1e-300));
    __syncthreads();
    for (int i = j + tid; i < nb; i += T) Vs[i][j] = (i == j) ? mk(piv, 0.0) : (1.0 / piv) * Vs[i][j];
    __syncthreads();
    for (int e = tid; e < nb * nb; e += T) {
      const int i = e % nb, k = e / nb;
      if (k > j && i >= k) Vs[i][k] = Vs[i][k] - Vs[i][j] * conj(Vs[k][j]);
    }
    __syncthreads();
  }
  cd *Lr = it.Lr;
  for (int e = tid; e < nb * nb; e += T) Lr[e] = Vs[e % nb][e / nb];
  __syncthreads();
  // H1 = L^-1 G (column c by thread c, in place)
  if (tid < nb) {
    const int c = tid;
    for (int i = 0; i < nb; ++i) {
      cd x = Gs[i][c];
      for (int k = 0; k < i; ++k) x = x - Vs[i][k] * Gs[k][c];
      Gs[i][c] = (1.0 / Vs[i][i].re) * x;
    }
  }
  __syncthreads();
  // G' = L^-1 H1^H into Vs (column c from the conjugated row c of H1); L is
  // read from Lr, so Vs can be overwritten column by column
  if (tid < nb) {
    const int c = tid;
    for (int i = 0; i < nb; ++i) {
      cd v = conj(Gs[c][i]);
      for (int k = 0; k < i; ++k) v = v - Lr[i + (size_t)k * nb] * Vs[k][c];
      Vs[i][c] = (1.0 / Lr[i + (size_t)i * nb].re) * v;
    }
  }
  __syncthreads();
  // Jacobi on G' (now Vs), eigenvectors accumulated in Gs (= I)
  for (int e = tid; e < nb * nb; e += T) {
    const int a = e % nb, b = e / nb;
    Gs[a][b] = mk(a == b ? 1.0 : 0.0, 0.0);
  }
  for (int e = tid; e < nb * nb; e += T) {
    const int a = e % nb, b = e / nb;
    if (a < b) {
      const cd x = Vs[a][b], y2 = Vs[b][a];
      const cd hm = mk(0.5 * (x.re + y2.re), 0.5 * (x.im - y2.im));
      Vs[a][b] = hm;
      Vs[b][a] = conj(hm);
    } else if (a == b) {
      Vs[a][a].im = 0.0;
    }
  }
  __syncthreads();
  jacobi_eig(Vs, Gs, nb, rc, rs, rph, pa, pb);
  // sort eigenvalues ascending
  if (tid == 0) {
    for (int a = 0; a < nb; ++a) { perm[a] = a; evs[a] = Vs[a][a].re; }
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
  // P = L^-H V: back substitution with L^H, column c by thread c (in place in Gs)
  if (tid < nb) {
    const int c = tid;
    for (int i = nb - 1; i >= 0; --i) {
      cd x = Gs[i][c];
      for (int k = i + 1; k < nb; ++k) x = x - conj(Lr[k + (size_t)i * nb]) * Gs[k][c];
      Gs[i][c] = (1.0 / Lr[i + (size_t)i * nb].re) * x;
    }
  }
  __syncthreads();
  const cd *Y = it.Y;
  cd *Z = it.Z;
  if (it.check) {
    // residuals of the refined pairs, R(:, b) = (C Y) p_b - theta_b Y p_b
    // (p_b = column perm[b] of P), into the free inverse-iteration scratch
    // before Z (= C Y) is overwritten; rr_product and rr_estimate take
    // them from there
    cd *Rv = (cd *)it.lu;
    for (size_t e = tid; e < (size_t)n * nb; e += T) {
      const int r = (int)(e % n), b = (int)(e / n);
      const int pbb = perm[b];
      const double th = evs[pbb];
      cd acc = mk(0.0, 0.0);
      for (int a = 0; a < nb; ++a)
        acc = cfma(gld(Z, (size_t)a * ld + r) - th * gld(Y, (size_t)a * ld + r), Gs[a][pbb], acc);
      gst(Rv, e, acc);
    }
    __syncthreads();
  } else if (tid == 0) {
    *it.acc = 0.0;
  }
  // Z = Y P(:, perm)
  for (size_t e = tid; e < (size_t)n * nb; e += T) {
    const int r = (int)(e % n), b = (int)(e / n);
    const int pbb = perm[b];
    cd acc = mk(0.0, 0.0);
    for (int a = 0; a < nb; ++a) acc = cfma(gld(Y, (size_t)a * ld + r), Gs[a][pbb], acc);
    gst(Z, (size_t)b * ld + r, acc);
  }
}

// Error estimate of the refined bands of an item with check set: with the
// residual r_b = C z_b - theta_b z_b of the unit Ritz vector z_b and its
// Rayleigh quotient rho_b = r_b^H C r_b / |r_b|^2, the second-order estimate
// e_b = |r_b|^2 / (rho_b - theta_b) of theta_b - lambda (the residual is
// orthogonal to the Ritz space, so rho_b - theta_b is its effective
// distance to the rest of the spectrum; |r_b| itself if rho_b <= theta_b),
// as a relative frequency error e_b / (2 theta_b), or e_b / (2 theta_top)
// below 1e-3 of the top frequency.  *acc = the largest over the bands.
__global__ void __launch_bounds__(64) rr_estimate(const EigItem *__restrict__ items) {
  const EigItem &it = items[blockIdx.x];
  if (!it.check) return;
  const int n = it.n, nb = it.nb, nrb = (n + 63) / 64;
  const double top = fmax(it.lam[nb - 1], 0.0);
  double worst = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) {
    double g = 0.0, m = 0.0;
    for (int q = 0; q < nrb; ++q) {
      const cd *P = it.Gp + (size_t)q * 2 * nb * nb;
      g += gld(P, (size_t)b * nb + b).re;
      m += gld(P, (size_t)nb * nb + (size_t)b * nb + b).re;
    }
    const double th = it.lam[b];
    double e = 0.0;
    if (m > 0.0) {
      const double rho = g / m;
      e = rho > th ? m / (rho - th) : sqrt(m);
    }
    const double den = 2.0 * (th >= 1e-6 * top ? th : top);
    const double est = (e == 0.0) ? 0.0 : (den > 0.0 ? e / den : INFINITY);
    worst = fmax(worst, est);
  }
  for (int o = 32; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o, 64));
  if (threadIdx.x == 0) *it.acc = worst;
}

// Bands per pass of the product kernel: the smallest of 8, 12, ..., 24 that
// holds every band in one pass (no products with padding columns beyond
// it), else passes of 24.
static const void *rr_product_fn(bool res, int nb) {
  static const void *const fns[2][5] = {
      {(const void *)rr_product<false, 8>, (const void *)rr_product<false, 12>, (const void *)rr_product<false, 16>,
       (const void *)rr_product<false, 20>, (const void *)rr_product<false, 24>},
      {(const void *)rr_product<true, 8>, (const void *)rr_product<true, 12>, (const void *)rr_product<true, 16>,
       (const void *)rr_product<true, 20>, (const void *)rr_product<true, 24>}};
  const int c = nb <= 8 ? 0 : (nb <= 12 ? 1 : (nb <= 16 ? 2 : (nb <= 20 ? 3 : 4)));
  return fns[res ? 1 : 0][c];
}

static void launch_rr_product(bool res, int nrb, int n_items, int nb, const EigItem *items, hipStream_t st) {
  const void *f = rr_product_fn(res, nb);
  void *args[] = {(void *)&items};
  (void)hipLaunchKernel(f, dim3(nrb, n_items), dim3(256), args, sizeof(cd) * 2 * 64 * nb, st);
}

hipError_t launch_rayleigh_ritz(const EigItem *items, int n_items, int n_max, int nb, bool check, hipStream_t st) {
  ProfScope ps(K_RR, st);
  const int nrb = (n_max + 63) / 64;
  launch_rr_product(false, nrb, n_items, nb, items, st);
  hipLaunchKernelGGL(rr_small, dim3(n_items), dim3(256), 0, st, items);
  if (check) {
    launch_rr_product(true, nrb, n_items, nb, items, st);
    hipLaunchKernelGGL(rr_estimate, dim3(n_items), dim3(64), 0, st, items);
  }
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) tridiag_results(const EigItem *__restrict__ items) {
  const EigItem &it = items[blockIdx.x];
  for (int b = threadIdx.x; b < it.nb; b += 256) {
    const double lam = it.lam_t[b];
    it.lam[b] = lam;
    it.omega[b] = sqrt(fmax(lam, 0.0));
  }
  if (threadIdx.x == 0) *it.acc = 0.0;
}

hipError_t launch_tridiag_results(const EigItem *items, int n_items, int nb, hipStream_t st) {
  (void)nb;
  hipLaunchKernelGGL(tridiag_results, dim3(n_items), dim3(256), 0, st, items);
  return hipGetLastError();
}

// Dynamic LDS above the default limit has to be opted into per kernel.
hipError_t init_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute((const void *)tridiag_bisect_item, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(double) * (3 * MAX_N + 1)));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)tridiag_twisted, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * 4 * MAX_N));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)tridiag_invit<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * 8 * INV_LDS_MAX_N));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)tridiag_invit<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * 3 * MAX_N));
  for (int res = 0; res < 2 && e == hipSuccess; ++res)
    for (int nb = 8; nb <= RRP_BC_MAX && e == hipSuccess; nb += 4)
      e = hipFuncSetAttribute(rr_product_fn(res != 0, nb), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(cd) * 2 * 64 * RR_MAX_BANDS));
  if (e != hipSuccess) return e;
  return init_band_attributes();
}

}  // namespace mvpb
