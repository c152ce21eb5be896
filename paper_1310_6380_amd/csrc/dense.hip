// Dense complex FP64 building blocks: Cholesky with explicit inverse of the
// factor (one workgroup per matrix) and a batched tiled GEMM.
#include "common.h"
#include "kernels.h"
#include "prof.h"

namespace mvpb {

// ---------------------------------------------------------------------------
// Cholesky A = L L^H (lower, in place) followed by X = L^-1 (lower).
// One 1024-thread workgroup per matrix; the current column of L (or row of
// X) is staged in LDS.  A right-looking rank-1 sweep per column: the
// per-cell factorisations are off the per-k hot path.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) potrf_trtri(cd *const *Aarr, cd *const *Xarr, int *status, int N) {
  extern __shared__ cd vec[];  // N entries
  __shared__ double piv_s;
  __shared__ int fail;
  cd *A = Aarr[blockIdx.x];
  cd *X = Xarr[blockIdx.x];
  const int tid = threadIdx.x, T = blockDim.x;
  const int lane = tid & 63, w = tid >> 6, nw = T >> 6;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < N; ++j) {
    if (tid == 0) {
      const double p = A[(size_t)j * N + j].re;
      if (!(p > 0.0) || !isfinite(p)) fail = j + 1;
      piv_s = sqrt(p);
    }
    __syncthreads();
    if (fail) break;
    const double s = piv_s, inv = 1.0 / s;
    for (int i = j + tid; i < N; i += T) {
      cd v = (i == j) ? mk(s, 0.0) : inv * A[(size_t)j * N + i];
      A[(size_t)j * N + i] = v;
      vec[i] = v;
    }
    __syncthreads();
    for (int k = j + 1 + w; k < N; k += nw) {
      const cd ck = conj(vec[k]);
      cd *colk = A + (size_t)k * N;
      for (int i = k + lane; i < N; i += 64) colk[i] = colk[i] - vec[i] * ck;
    }
    __syncthreads();
  }
  if (tid == 0) status[blockIdx.x] = fail;
  if (fail) return;
  // X = I
  for (size_t e = tid; e < (size_t)N * N; e += T) {
    const int r = (int)(e % N), c = (int)(e / N);
    X[e] = mk(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // forward substitution on all right-hand sides at once, row by row
  cd *rowk = vec;  // row k of X (columns 0..k)
  for (int k = 0; k < N; ++k) {
    const double inv = 1.0 / A[(size_t)k * N + k].re;
    for (int c = tid; c <= k; c += T) {
      const cd v = inv * X[(size_t)c * N + k];
      X[(size_t)c * N + k] = v;
      rowk[c] = v;
    }
    __syncthreads();
    const cd *Lk = A + (size_t)k * N;
    for (int c = w; c <= k; c += nw) {
      const cd xv = rowk[c];
      cd *colc = X + (size_t)c * N;
      for (int i = k + 1 + lane; i < N; i += 64) colc[i] = colc[i] - Lk[i] * xv;
    }
    __syncthreads();
  }
}

hipError_t launch_potrf_trtri(cd *const *A, cd *const *Linv, int *status, int count, int N, hipStream_t st) {
  ProfScope ps(K_POTRF, st);
  hipLaunchKernelGGL(potrf_trtri, dim3(count), dim3(1024), sizeof(cd) * N, st, A, Linv, status, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched complex GEMM, 64 x 64 tiles, 256 threads, 4 x 4 outputs per thread.
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
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  cd acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = mk(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    // A tile: 64 x 8
    for (int e = tid; e < BM * BK; e += 256) {
      int i, k;
      if (OPA == OP_N) { i = e % BM; k = e / BM; } else { k = e % BK; i = e / BK; }
      const int gi = m0 + i, gk = k0 + k;
      cd v = mk(0.0, 0.0);
      if (gi < M && gk < K) {
        v = (OPA == OP_N) ? A[(size_t)gk * bt.lda + gi] : conj(A[(size_t)gi * bt.lda + gk]);
        if (s) v = s[gk] * v;
      }
      As[k][i] = v;
    }
    // B tile: 8 x 64
    for (int e = tid; e < BK * BN; e += 256) {
      int k, j;
      if (OPB == OP_N) { k = e % BK; j = e / BK; } else { j = e % BN; k = e / BN; }
      const int gk = k0 + k, gj = n0 + j;
      cd v = mk(0.0, 0.0);
      if (gk < K && gj < N) v = (OPB == OP_N) ? B[(size_t)gj * bt.ldb + gk] : conj(B[(size_t)gk * bt.ldb + gj]);
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      cd av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tx + 16 * a];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][ty + 16 * c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = cfma(av[a], bv[c], acc[a][c]);
    }
    __syncthreads();
  }
  const bool use_beta = (beta.re != 0.0 || beta.im != 0.0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int gj = n0 + ty + 16 * c;
    if (gj >= N) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int gi = m0 + tx + 16 * a;
      if (gi >= M) continue;
      cd v = alpha * acc[a][c];
      cd *dst = C + (size_t)gj * bt.ldc + gi;
      if (use_beta) v = v + beta * (*dst);
      *dst = v;
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
