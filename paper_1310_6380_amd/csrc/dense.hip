// Dense complex FP64 building blocks: blocked Cholesky with the explicit
// inverse of the factor, and a batched tiled GEMM.
#include "common.h"
#include "kernels.h"
#include "prof.h"

#include <algorithm>

namespace mvpb {

// ---------------------------------------------------------------------------
// Cholesky A = L L^H (lower, in place) and X = L^-1 (lower, strict upper part
// zero) for a batch of N x N matrices, blocked by 64:
//   potrf_diag    factor of the diagonal block jb and its inverse (one
//                 workgroup per matrix, in LDS);
//   potrf_panel   L[i, jb] = A[i, jb] L_jj^-H for the row blocks below, and
//                 X[jb, c] = X_jj Y[jb, c] for the blocks c left of jb;
//   potrf_update  A[i, k] -= L[i, jb] L[k, jb]^H on the lower trailing tiles,
//                 and Y[i, c] -= L[i, jb] X[jb, c] for i below jb, c <= jb.
// Y[i, c] = -sum_{k=c}^{i-1} L[i, k] X[k, c] is built up in the blocks of X
// below the diagonal over the steps k (block forward substitution of
// L X = I), and X[i, c] = X_ii Y[i, c] once step i has the factor of block i.
// status[b] = j+1 if the pivot of column j of matrix b was not positive; the
// later launches skip that matrix.
// ---------------------------------------------------------------------------
constexpr int CB = 64;
typedef double zd4_t __attribute__((ext_vector_type(4)));

// D = A B for one 64 x 64 tile from LDS, D(r, c) = sum_{k < K} Ar[r][k] B(k, c)
// with B(k, c) = Bm[k][c] (TRB false) or conj(Bm[c][k]) (TRB true); entries
// with k >= K must be zero in both (K is rounded up to the 4-deep step).  On
// the FP64 matrix cores as D^T = B^T A^T, three real 16x16x4 products per
// complex step (Gauss: p1 = br ar, p2 = bi ai, p3 = (br + bi)(ar + ai)), so
// that a lane's results run down a column: wavefront wv owns columns
// 16 wv .. 16 wv + 15, and lane l holds D(16 rb + l % 16, 16 wv + l / 16 + 4 v)
// = (p1 - p2, p3 - p1 - p2)[rb][v].
template <bool TRB>
MVPB_DEV void tile_mfma(const cd (*Ar)[CB + 1], const cd (*Bm)[CB + 1], int K, zd4_t p1[4], zd4_t p2[4],
                        zd4_t p3[4]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) p1[rb] = p2[rb] = p3[rb] = zd4_t{0.0, 0.0, 0.0, 0.0};
  const int c = 16 * wv + li;
  for (int kk = 0; kk < K; kk += 4) {
    const int k = kk + lk;
    const cd bv = TRB ? conj(Bm[c][k]) : Bm[k][c];
    const double bs = bv.re + bv.im;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const cd av = Ar[16 * rb + li][k];
      p1[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv.re, av.re, p1[rb], 0, 0, 0);
      p2[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv.im, av.im, p2[rb], 0, 0, 0);
      p3[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(bs, av.re + av.im, p3[rb], 0, 0, 0);
    }
  }
}
MVPB_DEV cd tile_value(const zd4_t p1[4], const zd4_t p2[4], const zd4_t p3[4], int rb, int v) {
  return mk(p1[rb][v] - p2[rb][v], p3[rb][v] - p1[rb][v] - p2[rb][v]);
}

// Stage 64 x 64 tiles of column-major matrices into LDS: T[i][c0 + k] =
// M[idx] where where(i, k, idx) holds, else zero.  Thread t takes the entries
// e = t + 256 u (i = e % 64 fastest, so a wavefront reads one column run);
// every load is issued, from element 0 where masked, before the first LDS
// store, so that a thread's loads of both tiles are in flight together.
constexpr int STAGE_PER_THREAD = CB * CB / 256;
template <int W1, int W2, typename F1, typename F2>
MVPB_DEV void stage_tiles(cd (*T1)[W1], int c1, const cd *M1, F1 where1, cd (*T2)[W2], int c2, const cd *M2,
                          F2 where2) {
  cd v1[STAGE_PER_THREAD], v2[STAGE_PER_THREAD];
  bool o1[STAGE_PER_THREAD], o2[STAGE_PER_THREAD];
#pragma unroll
  for (int u = 0; u < STAGE_PER_THREAD; ++u) {
    const int e = threadIdx.x + 256 * u, i = e % CB, k = e / CB;
    size_t x1 = 0, x2 = 0;
    o1[u] = where1(i, k, x1);
    o2[u] = where2(i, k, x2);
    v1[u] = gld(M1, o1[u] ? x1 : 0);
    v2[u] = gld(M2, o2[u] ? x2 : 0);
  }
#pragma unroll
  for (int u = 0; u < STAGE_PER_THREAD; ++u) {
    const int e = threadIdx.x + 256 * u, i = e % CB, k = e / CB;
    T1[i][c1 + k] = o1[u] ? v1[u] : mk(0.0, 0.0);
    T2[i][c2 + k] = o2[u] ? v2[u] : mk(0.0, 0.0);
  }
}

// Factor and inverse of one diagonal block together: step j of the
// elimination scales column j of L and row j of the inverse, then updates
// the trailing lower triangle of the block and the rows of the inverse below
// j (forward elimination of [L | I]).  The diagonal of L is kept apart so that
// the pivot of the next step is read without a third barrier.  [Xi | L] sit
// side by side in one LDS array, so that in the update every lane (column c
// of [Xi | L]) does the same read-modify-write per row: of Xi for c <= j, of
// L for c > j (the upper triangle of L is updated too, never read).
__global__ void __launch_bounds__(256) potrf_diag(cd *const *Aarr, cd *const *Xarr, int *status, int N, int jb) {
  __shared__ cd DD[CB][2 * CB + 1];   // DD[r][c] = Xi[r][c], DD[r][CB + c] = L[r][c]
  __shared__ double dg[CB];
  __shared__ cd colj[CB];   // column j of L below the diagonal
  const int b = blockIdx.x;
  if (status[b]) return;
  cd *A = Aarr[b];
  cd *X = Xarr[b];
  const int nb = min(CB, N - jb);
  const int tid = threadIdx.x, c_ = tid & (CB - 1), w_ = tid / CB;
  const size_t ld = (size_t)N;
  {
    cd v[STAGE_PER_THREAD];
#pragma unroll
    for (int u = 0; u < STAGE_PER_THREAD; ++u) {
      const int e = tid + 256 * u, r = e % CB, c = e / CB;
      const bool ok = r < nb && c < nb && r >= c;
      v[u] = gld(A, ok ? (size_t)(jb + c) * ld + jb + r : 0);
    }
#pragma unroll
    for (int u = 0; u < STAGE_PER_THREAD; ++u) {
      const int e = tid + 256 * u, r = e % CB, c = e / CB;
      DD[r][CB + c] = (r < nb && c < nb && r >= c) ? v[u] : mk(0.0, 0.0);
      DD[r][c] = mk(r == c ? 1.0 : 0.0, 0.0);
    }
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double piv = DD[j][CB + j].re;
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (tid == 0) status[b] = jb + j + 1;
      return;   // uniform: every thread read the same pivot
    }
    const double sq = sqrt(piv), inv = 1.0 / sq;
    // column j of L below the diagonal, row j of the inverse (entries c <= j)
    if (tid < CB) {
      const int r = tid;
      if (r > j && r < nb) {
        const cd l = inv * DD[r][CB + j];
        DD[r][CB + j] = l;
        colj[r] = l;
      }
      if (r <= j) DD[j][r] = inv * DD[j][r];
      if (r == 0) dg[j] = sq;
    }
    __syncthreads();
    // lane = column c, wavefront w = rows r = w (mod 4) below j:
    // Xi[r][c] -= L[r][j] Xi[j][c] for c <= j; L[r][c] -= L[r][j] conj(L[c][j]) for c > j
    {
      const bool inv_col = c_ <= j;
      const int cc = inv_col ? c_ : CB + c_;
      const cd op = inv_col ? DD[j][c_] : conj(colj[c_]);
#pragma unroll 4
      for (int r = j + 1 + ((w_ - j - 1) & 3); r < nb; r += 4) DD[r][cc] = DD[r][cc] - colj[r] * op;
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e % nb, c = e / nb;
    if (r >= c) A[(size_t)(jb + c) * ld + jb + r] = (r == c) ? mk(dg[r], 0.0) : DD[r][CB + c];
    X[(size_t)(jb + c) * ld + jb + r] = (r >= c) ? DD[r][c] : mk(0.0, 0.0);
  }
}

// L[i0:i0+64, jb:jb+nb] = A[i0:i0+64, jb:jb+nb] X_jj^H
__global__ void __launch_bounds__(256) potrf_panel(cd *const *Aarr, cd *const *Xarr, const int *status, int N,
                                                    int jb) {
  __shared__ cd P[CB][CB + 1];    // P[r][k]
  __shared__ cd Di[CB][CB + 1];   // Di[c][k] = X_jj(c, k)
  const int b = blockIdx.y;
  if (status[b]) return;
  cd *A = Aarr[b];
  cd *X = Xarr[b];
  const int nb = min(CB, N - jb);
  const int m = N - jb - nb, rbn = m > 0 ? (m + CB - 1) / CB : 0;
  const size_t ldx = (size_t)N;
  if ((int)blockIdx.x >= rbn) {
    // X[jb, c-block] = X_jj Y[jb, c-block] in place (c-block left of jb, full
    // width); no other workgroup of the launch touches that block
    const int c0 = (blockIdx.x - rbn) * CB;
    const int tid = threadIdx.x, li = tid & 15, lk = (tid & 63) >> 4, wv = tid >> 6;
    // Di = X_jj (lower); P[k'][c] = Y[jb + k'][c0 + c]
    stage_tiles(
        Di, 0, X,
        [&](int r, int k, size_t &x) { x = (size_t)(jb + k) * ldx + jb + r; return r < nb && k < nb && r >= k; },
        P, 0, X, [&](int r, int k, size_t &x) { x = (size_t)(c0 + k) * ldx + jb + r; return r < nb; });
    __syncthreads();
    zd4_t p1[4], p2[4], p3[4];
    tile_mfma<false>(Di, P, nb, p1, p2, p3);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * rb + li, cc = 16 * wv + lk + 4 * v;
        if (r < nb) X[(size_t)(c0 + cc) * ldx + jb + r] = tile_value(p1, p2, p3, rb, v);
      }
    return;
  }
  const int i0 = jb + nb + blockIdx.x * CB;
  if (i0 >= N) return;
  const int rows = min(CB, N - i0);
  const size_t ld = (size_t)N;
  const int tid = threadIdx.x, li = tid & 15, lk = (tid & 63) >> 4, wv = tid >> 6;
  stage_tiles(
      P, 0, A, [&](int r, int k, size_t &x) { x = (size_t)(jb + k) * ld + i0 + r; return r < rows && k < nb; }, Di,
      0, X, [&](int r, int k, size_t &x) { x = (size_t)(jb + k) * ld + jb + r; return r < nb && k < nb && r >= k; });
  __syncthreads();
  zd4_t p1[4], p2[4], p3[4];
  tile_mfma<true>(P, Di, nb, p1, p2, p3);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * rb + li, cc = 16 * wv + lk + 4 * v;
      if (cc < nb && r < rows) A[(size_t)(jb + cc) * ld + i0 + r] = tile_value(p1, p2, p3, rb, v);
    }
}

MVPB_DEV int tri_row(int t) {   // I with I (I + 1) / 2 <= t < (I + 1) (I + 2) / 2
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  return I;
}

// A[i, k] -= L[i, jb] L[k, jb]^H on the lower 64 x 64 tiles right of jb+nb
__global__ void __launch_bounds__(256) potrf_update(cd *const *Aarr, cd *const *Xarr, const int *status, int N,
                                                     int jb) {
  __shared__ cd Lr[CB][CB + 1];   // Lr[r][k] = L(tile rows, jb+k)
  __shared__ cd Lc[CB][CB + 1];   // Lc[c][k] = L(tile cols, jb+k)
  const int b = blockIdx.y;
  if (status[b]) return;
  cd *A = Aarr[b];
  const int nb = min(CB, N - jb);
  const int q0 = jb + nb, m = N - q0;
  if (m <= 0) return;
  const int nt = (m + CB - 1) / CB;
  const int t = blockIdx.x;
  if (t >= nt * (nt + 1) / 2) {
    // Y[i-block, c-block] -= L[i-block, jb] X[jb, c-block] for the row blocks
    // i below jb and the column blocks c <= jb (the first contribution, c = jb,
    // is written without reading: Y starts at zero)
    const int jn = jb / CB + 1, t2 = t - nt * (nt + 1) / 2;
    const int I = t2 / jn, Cb = t2 % jn;
    if (I >= nt) return;
    cd *X = Xarr[b];
    const int r0 = q0 + I * CB, cx0 = Cb * CB;
    const bool first = cx0 == jb;
    const int cols = first ? nb : CB;
    const size_t ld = (size_t)N;
    const int tid = threadIdx.x, li = tid & 15, lk = (tid & 63) >> 4, wv = tid >> 6;
    // the entries this thread updates, loaded with the tiles (Y starts at zero)
    cd cur[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * rb + li, cc = 16 * wv + lk + 4 * v;
        const bool ok = !first && cc < cols && r < N;
        cur[rb][v] = gld(X, ok ? (size_t)(cx0 + cc) * ld + r : 0);
      }
    // Lr[i][k] = L[r0 + i][jb + k]; Lc[k'][c] = X[jb + k'][cx0 + c]
    stage_tiles(
        Lr, 0, A, [&](int i, int k, size_t &x) { x = (size_t)(jb + k) * ld + r0 + i; return r0 + i < N && k < nb; },
        Lc, 0, X, [&](int i, int k, size_t &x) { x = (size_t)(cx0 + k) * ld + jb + i; return k < cols && i < nb; });
    __syncthreads();
    zd4_t p1[4], p2[4], p3[4];
    tile_mfma<false>(Lr, Lc, nb, p1, p2, p3);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * rb + li, cc = 16 * wv + lk + 4 * v;
        if (cc < cols && r < N) {
          const cd c0v = first ? mk(0.0, 0.0) : cur[rb][v];
          X[(size_t)(cx0 + cc) * ld + r] = c0v - tile_value(p1, p2, p3, rb, v);
        }
      }
    return;
  }
  const int I = tri_row(t);
  const int J = t - I * (I + 1) / 2;
  const int r0 = q0 + I * CB, c0 = q0 + J * CB;
  const size_t ld = (size_t)N;
  const int tid = threadIdx.x, li = tid & 15, lk = (tid & 63) >> 4, wv = tid >> 6;
  // the entries this thread updates, loaded with the tiles
  cd cur[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 16 * rb + li, cc = c0 + 16 * wv + lk + 4 * v;
      const bool ok = cc < N && r < N && r >= cc;
      cur[rb][v] = gld(A, ok ? (size_t)cc * ld + r : 0);
    }
  stage_tiles(
      Lr, 0, A, [&](int i, int k, size_t &x) { x = (size_t)(jb + k) * ld + r0 + i; return r0 + i < N && k < nb; },
      Lc, 0, A, [&](int i, int k, size_t &x) { x = (size_t)(jb + k) * ld + c0 + i; return c0 + i < N && k < nb; });
  __syncthreads();
  zd4_t p1[4], p2[4], p3[4];
  tile_mfma<true>(Lr, Lc, nb, p1, p2, p3);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + 16 * rb + li, cc = c0 + 16 * wv + lk + 4 * v;
      if (cc < N && r < N && r >= cc) A[(size_t)cc * ld + r] = cur[rb][v] - tile_value(p1, p2, p3, rb, v);
    }
}

__global__ void zero_upper_blocks(cd *const *Xarr, const int *status, int N) {
  // strict upper block part of X (block rows above the diagonal block)
  const int b = blockIdx.y;
  if (status[b]) return;
  cd *X = Xarr[b];
  const size_t total = (size_t)N * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % N), c = (int)(e / N);
    if (r / CB < c / CB) X[e] = mk(0.0, 0.0);
  }
}

__global__ void clear_status(int *status, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) status[t] = 0;
}

// Inverse factors of the matrices whose factorisation stopped (status set)
// replaced by the identity, so that work which follows them in one launch
// sequence sees finite, well-conditioned input; the caller reports the
// failure from the status words.
__global__ void identity_if_failed(cd *const *Xarr, const int *status, int N) {
  const int b = blockIdx.y;
  if (!status[b]) return;
  cd *X = Xarr[b];
  const size_t total = (size_t)N * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % N), c = (int)(e / N);
    X[e] = mk(r == c ? 1.0 : 0.0, 0.0);
  }
}

hipError_t launch_identity_if_failed(cd *const *Linv, const int *status, int count, int N, hipStream_t st) {
  hipLaunchKernelGGL(identity_if_failed, dim3(64, count), dim3(256), 0, st, Linv, status, N);
  return hipGetLastError();
}

hipError_t launch_potrf_trtri(cd *const *A, cd *const *Linv, int *status, int count, int N, hipStream_t st) {
  ProfScope ps(K_POTRF, st);
  hipLaunchKernelGGL(clear_status, dim3((count + 255) / 256), dim3(256), 0, st, status, count);
  for (int jb = 0; jb < N; jb += CB) {
    const int nb = std::min(CB, N - jb), J = jb / CB;
    hipLaunchKernelGGL(potrf_diag, dim3(count), dim3(256), 0, st, A, Linv, status, N, jb);
    const int m = N - jb - nb, rb = m > 0 ? (m + CB - 1) / CB : 0;
    // panel tiles, then the J blocks of X left of the diagonal block
    if (rb + J > 0) hipLaunchKernelGGL(potrf_panel, dim3(rb + J, count), dim3(256), 0, st, A, Linv, status, N, jb);
    // trailing tiles, then rb (J + 1) tiles of the inverse
    if (m > 0)
      hipLaunchKernelGGL(potrf_update, dim3(rb * (rb + 1) / 2 + rb * (J + 1), count), dim3(256), 0, st, A, Linv,
                         status, N, jb);
  }
  hipLaunchKernelGGL(zero_upper_blocks, dim3(64, count), dim3(256), 0, st, Linv, status, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched complex GEMM, 64 x 64 tiles, 256 threads, on the FP64 matrix cores:
// wavefront wv owns tile rows 16 wv .. 16 wv + 15 and the four 16 x 16 column
// blocks.  Each complex step is three real 16x16x4 products (Gauss:
// p1 = ar br, p2 = ai bi, p3 = (ar + ai)(br + bi); re = p1 - p2,
// im = p3 - p1 - p2).  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of a 4-deep step and holds D[l / 16 + 4 v][l % 16].  (Deeper K tiles with
// the next tile prefetched into registers need more than 256 registers and
// halve the occupancy: slower.)
// ---------------------------------------------------------------------------
template <int OPA, int OPB>
__global__ void __launch_bounds__(256) zgemm_kernel(int M, int N, int K, cd alpha, GemmBatch bt, cd beta) {
  constexpr int BM = 64, BN = 64, BK = 8;
  __shared__ cd As[BK][BM + 1];
  __shared__ cd Bs[BK][BN + 1];
  const int b = blockIdx.z;
  const cd *__restrict__ A = bt.A[b];
  const cd *__restrict__ B = bt.B[b];
  cd *__restrict__ C = bt.C[b];
  const double *__restrict__ s = bt.s ? bt.s[b] : nullptr;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ai = lane & 15, ak = lane >> 4;
  zd4_t p1[4], p2[4], p3[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) p1[c] = p2[c] = p3[c] = zd4_t{0.0, 0.0, 0.0, 0.0};
  constexpr int PA = BM * BK / 256, PB = BK * BN / 256;   // tile entries per thread
  // the loads of step k0 + BK are issued right after the LDS stores of step
  // k0, so that they are in flight during its matrix-core products; every
  // load of a step is issued, from element 0 where masked, before the first
  // LDS store that waits for it
  cd va[PA], vb[PB];
  double sa[PA];
  bool oa[PA], ob[PB];
  auto load_step = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int e = tid + 256 * u;
      const int i = (OPA == OP_N) ? e % BM : e / BK, k = (OPA == OP_N) ? e / BM : e % BK;
      const int gi = m0 + i, gk = k0 + k;
      oa[u] = gi < M && gk < K;
      va[u] = gld(A, oa[u] ? ((OPA == OP_N) ? (size_t)gk * bt.lda + gi : (size_t)gi * bt.lda + gk) : 0);
      sa[u] = s ? gld(s, oa[u] ? (size_t)gk : 0) : 1.0;
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + 256 * u;
      const int k = (OPB == OP_N) ? e % BK : e / BN, j = (OPB == OP_N) ? e / BK : e % BN;
      const int gk = k0 + k, gj = n0 + j;
      ob[u] = gk < K && gj < N;
      vb[u] = gld(B, ob[u] ? ((OPB == OP_N) ? (size_t)gj * bt.ldb + gk : (size_t)gk * bt.ldb + gj) : 0);
    }
  };
  load_step(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int e = tid + 256 * u;
      const int i = (OPA == OP_N) ? e % BM : e / BK, k = (OPA == OP_N) ? e / BM : e % BK;
      const cd v = (OPA == OP_N) ? va[u] : conj(va[u]);
      As[k][i] = oa[u] ? (s ? sa[u] * v : v) : mk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + 256 * u;
      const int k = (OPB == OP_N) ? e % BK : e / BN, j = (OPB == OP_N) ? e / BK : e % BN;
      Bs[k][j] = ob[u] ? ((OPB == OP_N) ? vb[u] : conj(vb[u])) : mk(0.0, 0.0);
    }
    __syncthreads();
    if (k0 + BK < K) load_step(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const cd av = As[kk + ak][16 * wv + ai];
      const double as = av.re + av.im;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const cd bv = Bs[kk + ak][16 * c + ai];
        p1[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, p1[c], 0, 0, 0);
        p2[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.im, p2[c], 0, 0, 0);
        p3[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, bv.re + bv.im, p3[c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const bool use_beta = (beta.re != 0.0 || beta.im != 0.0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int gj = n0 + 16 * c + ai;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = m0 + 16 * wv + ak + 4 * v;
      if (gj >= N || gi >= M) continue;
      cd x = alpha * mk(p1[c][v] - p2[c][v], p3[c][v] - p1[c][v] - p2[c][v]);
      cd *dst = C + (size_t)gj * bt.ldc + gi;
      if (use_beta) x = x + beta * (*dst);
      *dst = x;
    }
  }
}

hipError_t launch_zgemm(Op opA, Op opB, int M, int N, int K, cd alpha, GemmBatch bt, cd beta, int count,
                        hipStream_t st) {
  dim3 grid((M + 63) / 64, (N + 63) / 64, count);
  ProfScope ps(K_GEMM, st);
  if (opA == OP_N && opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_N>), grid, dim3(256), 0, st, M, N, K, alpha, bt, beta);
  else if (opA == OP_N && opB == OP_C)
    hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C>), grid, dim3(256), 0, st, M, N, K, alpha, bt, beta);
  else if (opA == OP_C && opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_N>), grid, dim3(256), 0, st, M, N, K, alpha, bt, beta);
  else
    hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_C>), grid, dim3(256), 0, st, M, N, K, alpha, bt, beta);
  return hipGetLastError();
}

}  // namespace mvpb
