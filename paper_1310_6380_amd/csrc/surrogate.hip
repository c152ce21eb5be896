// Learned screening surrogate: a small periodic CNN that maps a binary
// 32 x 32 pixel cell to its lowest 10 bands at 40 k-points (normalised
// frequencies), trained on bands computed by the method itself.
//
//   conv1 3x3  1->32 s1, conv2..4 3x3 32->32 s2 (circular padding, ReLU)
//   flatten 4x4x32 = 512 -> fc1 256 (ReLU) -> fc2 400, mean squared error.
//
// Activations are NHWC FP32; a convolution is one GEMM whose A operand is
// the implicit im2col of its input (the tile loads gather the taps straight
// from the activations, circular padding, power-of-two grids), also for the
// weight gradients; the backward data pass is a GEMM into a column buffer
// and a gather col2im (every input pixel collects its taps, so no atomics
// and bitwise-reproducible results).  GEMMs run either as FP32 FMA
// tiles or on the matrix cores with BF16 inputs and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16), bias and ReLU applied in the GEMM epilogue,
// long reductions split over workgroups; master weights and Adam moments
// stay FP32.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../../include/mvpb.h"
#include "common.h"
#include "kernels.h"

namespace mvpb {

// ---------------------------------------------------------------------------
// GEMM, row-major: C[M x N] = act(alpha op(A) op(B) + beta C + bias).
// op(A) = A (A[i*lda+k]) or A^T (A[k*lda+i]); op(B) = B (B[k*ldb+j]) or B^T (B[j*ldb+k]).
// Long reductions (the weight gradients of the convolutions sum over every
// output pixel of the batch) are split over blockIdx.z: split z sums its K
// range into its own slice of a partial buffer, and gemm_reduce adds the
// slices in a fixed order (reproducible), applying alpha, beta and bias.
// ---------------------------------------------------------------------------
constexpr int GBM = 64, GBN = 64;

// Implicit im2col operand: column matrix col[p][k], p = (b, oy, ox) an output
// pixel, k = (ky 3 + kx) C + c, col[p][k] = in[b][(s oy + ky - 1) mod H]
// [(s ox + kx - 1) mod W][c] with H, W, C and the output grid Ho = H / s,
// Wo = W / s powers of two (given as log2).
struct ConvA {
  const float *in = nullptr;   // NHWC input; nullptr: A is an ordinary matrix
  int lH = 0, lW = 0, lC = 0, lHo = 0, lWo = 0, s = 1;
};
MVPB_DEV size_t conv_index(const ConvA &cv, int p, int k) {   // of col[p][k] in the input
  const int c = k & ((1 << cv.lC) - 1), tap = k >> cv.lC;
  const int ky = tap / 3, kx = tap - 3 * ky;
  const int ox = p & ((1 << cv.lWo) - 1), t = p >> cv.lWo;
  const int oy = t & ((1 << cv.lHo) - 1), b = t >> cv.lHo;
  const int y = (cv.s * oy + ky - 1) & ((1 << cv.lH) - 1), x = (cv.s * ox + kx - 1) & ((1 << cv.lW) - 1);
  return (((((size_t)b << cv.lH) + y) << cv.lW) + x) << cv.lC | (size_t)c;
}

struct GemmArgs {
  int M, N, K;
  float alpha, beta;
  const float *A;   // unused when conv.in is set (op(A) is then the implicit column matrix)
  int lda;
  const float *B;
  int ldb;
  float *C;          // output, or the partial buffer [splits][M][N] when kchunk < K
  int ldc;
  int kchunk;        // K range of one split
  const float *bias; // per column, nullable (applied when not split)
  int relu;
  ConvA conv;
};

// Every load of a thread is issued, from element 0 where masked, before its
// first LDS store, so that all of them are in flight together.
template <int TA, int TB, int BK>
MVPB_DEV void load_tiles(const GemmArgs &g, int m0, int n0, int k0, int k1, float (&As)[BK][GBM + 4],
                         float (&Bs)[BK][GBN + 4]) {
  constexpr int PA = GBM * BK / 256, PB = BK * GBN / 256;
  static_assert(PA * 256 == GBM * BK && PB * 256 == BK * GBN, "tile entries per thread");
  const int tid = threadIdx.x;
  float va[PA], vb[PB];
  bool oa[PA], ob[PB];
#pragma unroll
  for (int u = 0; u < PA; ++u) {
    const int e = tid + 256 * u;
    const int i = TA == 0 ? e / BK : e % GBM, k = TA == 0 ? e % BK : e / GBM;
    const int gi = m0 + i, gk = k0 + k;
    oa[u] = gi < g.M && gk < k1;
    if (g.conv.in) {   // op(A)[gi][gk] = col[gi][gk] (TA = 0) or col[gk][gi] (TA = 1)
      const size_t x = TA == 0 ? conv_index(g.conv, gi, gk) : conv_index(g.conv, gk, gi);
      va[u] = gld(g.conv.in, oa[u] ? x : 0);
    } else {
      const size_t x = TA == 0 ? (size_t)gi * g.lda + gk : (size_t)gk * g.lda + gi;
      va[u] = gld(g.A, oa[u] ? x : 0);
    }
  }
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int e = tid + 256 * u;
    const int k = TB == 0 ? e / GBN : e % BK, j = TB == 0 ? e % GBN : e / BK;
    const int gk = k0 + k, gj = n0 + j;
    ob[u] = gk < k1 && gj < g.N;
    vb[u] = gld(g.B, ob[u] ? (TB == 0 ? (size_t)gk * g.ldb + gj : (size_t)gj * g.ldb + gk) : 0);
  }
#pragma unroll
  for (int u = 0; u < PA; ++u) {
    const int e = tid + 256 * u;
    const int i = TA == 0 ? e / BK : e % GBM, k = TA == 0 ? e % BK : e / GBM;
    As[k][i] = oa[u] ? va[u] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int e = tid + 256 * u;
    const int k = TB == 0 ? e / GBN : e % BK, j = TB == 0 ? e % GBN : e / BK;
    Bs[k][j] = ob[u] ? vb[u] : 0.f;
  }
}

// Store one result: straight (with alpha, beta, the column's bias bj, ReLU)
// or into the split's partial slice.
MVPB_DEV void gemm_store(const GemmArgs &g, int i, int j, float acc, float bj) {
  if (i >= g.M || j >= g.N) return;
  if (g.kchunk < g.K) {
    g.C[((size_t)blockIdx.z * g.M + i) * g.N + j] = acc;
    return;
  }
  float *c = g.C + (size_t)i * g.ldc + j;
  float v = g.alpha * acc + (g.beta != 0.f ? g.beta * *c : 0.f) + bj;
  *c = g.relu ? fmaxf(v, 0.f) : v;
}
// Bias of column j (zero without bias or for a split), loaded from an
// in-range address so that a thread's loads are in flight together.
MVPB_DEV float gemm_bias(const GemmArgs &g, int j) {
  if (!g.bias || g.kchunk < g.K) return 0.f;   // uniform
  const float b = gld(g.bias, j < g.N ? (size_t)j : 0);
  return j < g.N ? b : 0.f;
}

template <int TA, int TB>
__global__ void __launch_bounds__(256) sgemm_f32(GemmArgs g) {
  constexpr int BK = 16;
  __shared__ float As[BK][GBM + 4];
  __shared__ float Bs[BK][GBN + 4];
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += BK) {
    load_tiles<TA, TB, BK>(g, m0, n0, k0, ke, As, Bs);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[kk][ty + 16 * q];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[kk][tx + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fmaf(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
  float bj[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) bj[q] = gemm_bias(g, n0 + tx + 16 * q);
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) gemm_store(g, m0 + ty + 16 * p, n0 + tx + 16 * q, acc[p][q], bj[q]);
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// Matrix-core GEMM: 64 x 64 block tile, 4 wavefronts of 32 x 32 (2 x 2
// v_mfma_f32_16x16x32_bf16 tiles, 32-deep K steps).  Lane l feeds
// A[row = l%16][k = 8(l/16)+v] and B[k = 8(l/16)+v][col = l%16], v < 8, and
// receives D[4(l/16)+v][l%16], v < 4.  Inputs are rounded to BF16 (nearest
// even) when they leave LDS; accumulation is FP32.
template <int TA, int TB>
__global__ void __launch_bounds__(256) sgemm_bf16(GemmArgs g) {
  constexpr int BK = 32;
  __shared__ float As[BK][GBM + 4];
  __shared__ float Bs[BK][GBN + 4];
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += BK) {
    load_tiles<TA, TB, BK>(g, m0, n0, k0, ke, As, Bs);
    __syncthreads();
    bf8v af[2], bf[2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int v = 0; v < 8; ++v) af[p][v] = (__bf16)As[8 * (lane >> 4) + v][wr + 16 * p + (lane & 15)];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 8; ++v) bf[q][v] = (__bf16)Bs[8 * (lane >> 4) + v][wc + 16 * q + (lane & 15)];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[p], bf[q], acc[p][q], 0, 0, 0);
    __syncthreads();
  }
  float bj[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) bj[q] = gemm_bias(g, n0 + wc + 16 * q + (lane & 15));
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        gemm_store(g, m0 + wr + 16 * p + 4 * (lane >> 4) + v, n0 + wc + 16 * q + (lane & 15), acc[p][q][v], bj[q]);
}

// C = act(alpha sum_z P[z] + beta C + bias), slices added in order z = 0, 1, ...
__global__ void __launch_bounds__(256) gemm_reduce(const float *__restrict__ P, int splits, int M, int N, float alpha,
                                                   float beta, float *__restrict__ C, int ldc,
                                                   const float *__restrict__ bias, int relu) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const int i = e / N, j = e % N;
  // eight slices' loads in flight at a time, added in slice order
  constexpr int U = 8;
  const size_t MN = (size_t)M * N;
  float acc = 0.f;
  int z = 0;
  for (; z + U <= splits; z += U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = gld(P, (size_t)(z + u) * MN + e);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  for (; z < splits; ++z) acc += P[(size_t)z * MN + e];
  float *c = C + (size_t)i * ldc + j;
  float v = alpha * acc + (beta != 0.f ? beta * *c : 0.f) + (bias ? bias[j] : 0.f);
  *c = relu ? fmaxf(v, 0.f) : v;
}

// Split K so that every output tile gets enough workgroups: long reductions
// (K >= 4096) are cut into chunks of at least 1024, at most 128 chunks, and
// only while the output tiles alone leave the chip idle.
static int gemm_splits(int M, int N, int K) {
  const long tiles = (long)((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
  if (K < 4096 || tiles >= 256) return 1;
  int sp = (int)std::min<long>(128, (512 + tiles - 1) / tiles);
  sp = std::min(sp, std::max(1, K / 1024));
  return sp;
}

static hipError_t gemm(bool bf16, int ta, int tb, int M, int N, int K, float alpha, const float *A, int lda,
                       const float *B, int ldb, float beta, float *C, int ldc, hipStream_t st,
                       const float *bias = nullptr, int relu = 0, float *split_buf = nullptr,
                       size_t split_cap = 0, const ConvA &conv = ConvA()) {
  int sp = gemm_splits(M, N, K);
  if ((size_t)sp * M * N > split_cap || !split_buf) sp = 1;
  const int align = bf16 ? 32 : 16;
  const int kchunk = sp == 1 ? K : ((K + sp - 1) / sp + align - 1) / align * align;
  sp = (K + kchunk - 1) / kchunk;
  GemmArgs g{M, N, K, alpha, beta, A, lda, B, ldb, sp == 1 ? C : split_buf, ldc, kchunk, bias, relu, conv};
  dim3 grid((N + GBN - 1) / GBN, (M + GBM - 1) / GBM, sp);
#define MVPB_GEMM_CASE(TA, TB)                                                            \
  if (ta == TA && tb == TB) {                                                             \
    if (bf16)                                                                             \
      hipLaunchKernelGGL((sgemm_bf16<TA, TB>), grid, dim3(256), 0, st, g);                \
    else                                                                                  \
      hipLaunchKernelGGL((sgemm_f32<TA, TB>), grid, dim3(256), 0, st, g);                 \
  }
  MVPB_GEMM_CASE(0, 0)
  MVPB_GEMM_CASE(0, 1)
  MVPB_GEMM_CASE(1, 0)
  MVPB_GEMM_CASE(1, 1)
#undef MVPB_GEMM_CASE
  if (sp > 1)
    hipLaunchKernelGGL(gemm_reduce, dim3((M * N + 255) / 256), dim3(256), 0, st, split_buf, sp, M, N, alpha, beta, C,
                       ldc, bias, relu);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Elementwise and reduction kernels
// ---------------------------------------------------------------------------
__global__ void cells_to_float(const uint8_t *__restrict__ cells, float *__restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = cells[i] ? 1.f : 0.f;
}

// Gather form of col2im: da[b][y][x][c] = sum over taps of dcol at the output
// pixel that reads (y, x) through that tap (if any).
__global__ void col2im(const float *__restrict__ dcol, float *__restrict__ da, int B, int H, int W, int C, int s) {
  const int Ho = H / s, Wo = W / s, K = 9 * C;
  const size_t total = (size_t)B * H * W * C;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const size_t pix = e / C;
    const int x = (int)(pix % W), y = (int)((pix / W) % H), b = (int)(pix / ((size_t)W * H));
    float acc = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
      const int ty = (y - ky + 1 + H) % H;
      if (ty % s) continue;
      const int oy = ty / s;
      for (int kx = 0; kx < 3; ++kx) {
        const int tx = (x - kx + 1 + W) % W;
        if (tx % s) continue;
        const int ox = tx / s;
        const size_t p = ((size_t)b * Ho + oy) * Wo + ox;
        acc += dcol[p * K + (ky * 3 + kx) * C + c];
      }
    }
    da[e] = acc;
  }
}

__global__ void relu_mask(float *__restrict__ d, const float *__restrict__ a, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    if (!(a[e] > 0.f)) d[e] = 0.f;
}

// Partial column sums: block (x, y) sums rows y, y + gridDim.y, ... of the
// 64-column slab x into part[y][c]; column_sums_fin adds the parts in order.
__global__ void __launch_bounds__(256) column_sums(const float *__restrict__ d, size_t rows, int C,
                                                   float *__restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  float acc = 0.f;
  if (c < C) {
    // eight rows' loads in flight at a time, added in row order
    constexpr int U = 8;
    const size_t r0 = (size_t)blockIdx.y * 4 + g, step = (size_t)gridDim.y * 4;
    size_t r = r0;
    for (; r + (U - 1) * step < rows; r += U * step) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = gld(d, (r + u * step) * C + c);
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u];
    }
    for (; r < rows; r += step) acc += d[r * C + c];
  }
  red[g][threadIdx.x & 63] = acc;
  __syncthreads();
  if (g == 0 && c < C) part[(size_t)blockIdx.y * C + c] = red[0][threadIdx.x] + red[1][threadIdx.x] +
                                                           red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void column_sums_fin(const float *__restrict__ part, int parts, int C, float *__restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  // eight parts' loads in flight at a time, added in part order
  constexpr int U = 8;
  float acc = 0.f;
  int p = 0;
  for (; p + U <= parts; p += U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = gld(part, (size_t)(p + u) * C + c);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u];
  }
  for (; p < parts; ++p) acc += part[(size_t)p * C + c];
  db[c] = acc;
}

// dout = 2 (out - y) / n and per-block partial sums of (out - y)^2
__global__ void __launch_bounds__(256) mse_grad(const float *__restrict__ out, const float *__restrict__ y, int n,
                                                float *__restrict__ dout, float *__restrict__ partial) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const float r = out[e] - y[e];
    dout[e] = 2.f * r / (float)n;
    acc += r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void adam_step(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                          int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void init_uniform(float *__restrict__ p, int n, float lim, unsigned long long seed, unsigned long long offset) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // counter-based hash (splitmix64 finaliser) -> uniform in [-lim, lim)
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (offset + i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const float u = (float)((z >> 40) * (1.0 / 16777216.0));
  p[i] = (2.f * u - 1.f) * lim;
}

}  // namespace mvpb

using namespace mvpb;

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

struct Layer {
  int ci, co, s, H, W;  // input H, W
};
const Layer kConv[4] = {{1, 32, 1, 32, 32}, {32, 32, 2, 32, 32}, {32, 32, 2, 16, 16}, {32, 32, 2, 8, 8}};
constexpr int kFcIn = 512, kFcHid = 256, kOut = 400, kPix = 32 * 32;
constexpr size_t kSplitCap = (size_t)2 << 20;   // floats of split-K partial slices
constexpr int kColParts = 256;                  // row blocks of the bias-gradient sums

int param_offsets(int *off) {  // 12 tensors
  int o = 0, t = 0;
  for (int l = 0; l < 4; ++l) {
    off[t++] = o;
    o += 9 * kConv[l].ci * kConv[l].co;
    off[t++] = o;
    o += kConv[l].co;
  }
  off[t++] = o;
  o += kFcIn * kFcHid;
  off[t++] = o;
  o += kFcHid;
  off[t++] = o;
  o += kFcHid * kOut;
  off[t++] = o;
  o += kOut;
  return o;
}

template <typename T>
struct Buf {
  T *p = nullptr;
  size_t n = 0;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t count) {
    n = count;
    return hipMalloc(&p, sizeof(T) * count);
  }
};

}  // namespace

struct mvpb_sur_s {
  mvpb_ctx ctx = nullptr;
  hipStream_t st = nullptr;
  int max_batch = 0;
  bool bf16 = true;
  int n_params = 0;
  int off[12];
  long long step = 0;
  uint64_t seed = 0;
  Buf<float> params, grads, m, v;
  Buf<float> act[5];        // act[0] input [B,32,32,1]; act[l+1] output of conv l (NHWC)
  Buf<float> dcol, dact, dact2;
  Buf<float> h, out, dout, dh, dflat, partial;
  Buf<float> split;     // partial slices of split-K GEMMs
  Buf<float> colpart;   // partial column sums (bias gradients)
  Buf<uint8_t> cells;
  Buf<float> target;
};

extern "C" int mvpb_sur_destroy(mvpb_sur net);

// GEMM with the network's precision and split-K scratch.
static hipError_t net_gemm(mvpb_sur net, int ta, int tb, int M, int N, int K, const float *A, int lda, const float *B,
                           int ldb, float *C, int ldc, const float *bias = nullptr, int relu = 0,
                           const ConvA &conv = ConvA()) {
  return gemm(net->bf16, ta, tb, M, N, K, 1.f, A, lda, B, ldb, 0.f, C, ldc, net->st, bias, relu, net->split.p,
              net->split.n, conv);
}

static int ilog2_exact(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// The implicit column matrix of conv layer L over the activations `in`.
static ConvA conv_operand(const Layer &L, const float *in) {
  ConvA cv;
  cv.in = in;
  cv.lH = ilog2_exact(L.H);
  cv.lW = ilog2_exact(L.W);
  cv.lC = ilog2_exact(L.ci);
  cv.lHo = ilog2_exact(L.H / L.s);
  cv.lWo = ilog2_exact(L.W / L.s);
  cv.s = L.s;
  return cv;
}

// db[c] = sum over rows of d[r][c] (blocks of rows, then the blocks in order).
static void col_sums(mvpb_sur net, const float *d, size_t rows, int C, float *db) {
  const int parts = (int)std::min<size_t>(kColParts, (rows + 511) / 512);
  hipLaunchKernelGGL(column_sums, dim3((C + 63) / 64, parts), dim3(256), 0, net->st, d, rows, C, net->colpart.p);
  hipLaunchKernelGGL(column_sums_fin, dim3((C + 255) / 256), dim3(256), 0, net->st, net->colpart.p, parts, C, db);
}

static int sur_forward(mvpb_sur net, int B) {
  hipStream_t st = net->st;
  float *P = net->params.p;
  hipError_t e = hipSuccess;
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    const Layer &L = kConv[l];
    const int Ho = L.H / L.s, Wo = L.W / L.s;
    const size_t rows = (size_t)B * Ho * Wo;
    const int K = 9 * L.ci;
    // convolution as one GEMM over the implicit column matrix, bias and ReLU in its epilogue
    e = net_gemm(net, 0, 0, (int)rows, L.co, K, nullptr, K, P + net->off[2 * l], L.co, net->act[l + 1].p, L.co,
                 P + net->off[2 * l + 1], 1, conv_operand(L, net->act[l].p));
  }
  // fc1 (ReLU), fc2
  if (e == hipSuccess)
    e = net_gemm(net, 0, 0, B, kFcHid, kFcIn, net->act[4].p, kFcIn, P + net->off[8], kFcHid, net->h.p, kFcHid,
                 P + net->off[9], 1);
  if (e == hipSuccess)
    e = net_gemm(net, 0, 0, B, kOut, kFcHid, net->h.p, kFcHid, P + net->off[10], kOut, net->out.p, kOut,
                 P + net->off[11], 0);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "surrogate forward: %s", hipGetErrorString(e));
  return MVPB_OK;
}

// Backward from net->dout; gradients into net->grads.
static int sur_backward(mvpb_sur net, int B) {
  hipStream_t st = net->st;
  float *P = net->params.p, *G = net->grads.p;
  hipError_t e = net_gemm(net, 1, 0, kFcHid, kOut, B, net->h.p, kFcHid, net->dout.p, kOut, G + net->off[10], kOut);
  col_sums(net, net->dout.p, (size_t)B, kOut, G + net->off[11]);
  if (e == hipSuccess) e = net_gemm(net, 0, 1, B, kFcHid, kOut, net->dout.p, kOut, P + net->off[10], kOut, net->dh.p, kFcHid);
  hipLaunchKernelGGL(relu_mask, dim3((B * kFcHid + 255) / 256), dim3(256), 0, st, net->dh.p, net->h.p, (size_t)B * kFcHid);
  if (e == hipSuccess)
    e = net_gemm(net, 1, 0, kFcIn, kFcHid, B, net->act[4].p, kFcIn, net->dh.p, kFcHid, G + net->off[8], kFcHid);
  col_sums(net, net->dh.p, (size_t)B, kFcHid, G + net->off[9]);
  if (e == hipSuccess)
    e = net_gemm(net, 0, 1, B, kFcIn, kFcHid, net->dh.p, kFcHid, P + net->off[8], kFcHid, net->dact.p, kFcIn);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "surrogate backward: %s", hipGetErrorString(e));
  float *da = net->dact.p, *da_next = net->dact2.p;
  for (int l = 3; l >= 0; --l) {
    const Layer &L = kConv[l];
    const int Ho = L.H / L.s, Wo = L.W / L.s;
    const size_t rows = (size_t)B * Ho * Wo;
    const int K = 9 * L.ci;
    // dz = da * relu'(act[l+1])
    hipLaunchKernelGGL(relu_mask, dim3((unsigned)std::min<size_t>((rows * L.co + 255) / 256, 65535)), dim3(256), 0, st,
                       da, net->act[l + 1].p, rows * L.co);
    // dW = col^T dz over the implicit column matrix (split over the output pixels), db = column sums of dz
    e = net_gemm(net, 1, 0, K, L.co, (int)rows, nullptr, K, da, L.co, G + net->off[2 * l], L.co, nullptr, 0,
                 conv_operand(L, net->act[l].p));
    col_sums(net, da, rows, L.co, G + net->off[2 * l + 1]);
    if (l > 0 && e == hipSuccess) {
      // dcol = dz W^T, then gather back onto the input pixels
      e = net_gemm(net, 0, 1, (int)rows, K, L.co, da, L.co, P + net->off[2 * l], L.co, net->dcol.p, K);
      const size_t tin = (size_t)B * L.H * L.W * L.ci;
      hipLaunchKernelGGL(col2im, dim3((unsigned)std::min<size_t>((tin + 255) / 256, 65535)), dim3(256), 0, st,
                         net->dcol.p, da_next, B, L.H, L.W, L.ci, L.s);
      float *t = da;
      da = da_next;
      da_next = t;
    }
    if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "surrogate backward: %s", hipGetErrorString(e));
  }
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "surrogate backward: %s", hipGetErrorString(e));
  return MVPB_OK;
}

static int stage_inputs(mvpb_sur net, int B, const uint8_t *cells, const float *target, unsigned flags,
                        const float **tgt_dev) {
  const bool dev = flags & MVPB_F_DEVICE_PTRS;
  const uint8_t *c = cells;
  if (!dev) {
    hipError_t e = hipMemcpyAsync(net->cells.p, cells, (size_t)B * kPix, hipMemcpyHostToDevice, net->st);
    if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "upload: %s", hipGetErrorString(e));
    c = net->cells.p;
  }
  hipLaunchKernelGGL(cells_to_float, dim3((B * kPix + 255) / 256), dim3(256), 0, net->st, c, net->act[0].p, B * kPix);
  if (target) {
    if (!dev) {
      hipError_t e = hipMemcpyAsync(net->target.p, target, sizeof(float) * B * kOut, hipMemcpyHostToDevice, net->st);
      if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "upload: %s", hipGetErrorString(e));
      *tgt_dev = net->target.p;
    } else {
      *tgt_dev = target;
    }
  }
  return MVPB_OK;
}

static int loss_and_grad_out(mvpb_sur net, int B, const float *tgt, float *loss) {
  const int n = B * kOut, nblk = 64;
  hipLaunchKernelGGL(mse_grad, dim3(nblk), dim3(256), 0, net->st, net->out.p, tgt, n, net->dout.p, net->partial.p);
  float part[64];
  hipError_t e = hipMemcpyAsync(part, net->partial.p, sizeof part, hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "loss: %s", hipGetErrorString(e));
  double s = 0.0;
  for (int i = 0; i < nblk; ++i) s += part[i];
  if (loss) *loss = (float)(s / n);
  return MVPB_OK;
}

extern "C" int mvpb_sur_create(mvpb_ctx ctx, int max_batch, int precision, uint64_t seed, mvpb_sur *out) {
  if (!ctx || !out) return set_error(MVPB_E_INVALID, "NULL argument");
  if (ctx_closing(ctx)) return set_error(MVPB_E_INVALID, "context has been destroyed");
  if (max_batch < 1 || max_batch > 65536) return set_error(MVPB_E_INVALID, "max_batch out of range");
  if (precision != 0 && precision != 1) return set_error(MVPB_E_INVALID, "precision must be 0 (FP32) or 1 (BF16)");
  (void)hipSetDevice(ctx_device(ctx));
  mvpb_sur net = new mvpb_sur_s();
  net->ctx = ctx;
  net->st = ctx_stream(ctx);
  net->max_batch = max_batch;
  net->bf16 = precision == 1;
  net->seed = seed;
  net->n_params = param_offsets(net->off);
  const size_t B = max_batch;
  size_t colmax = 0, actmax = 0;
  for (int l = 0; l < 4; ++l) {
    const Layer &L = kConv[l];
    colmax = std::max(colmax, B * (L.H / L.s) * (L.W / L.s) * 9 * L.ci);
    actmax = std::max(actmax, B * L.H * L.W * L.ci);
    actmax = std::max(actmax, B * (L.H / L.s) * (L.W / L.s) * L.co);
  }
  hipError_t e = hipSuccess;
  auto A = [&](Buf<float> &b, size_t n) {
    if (e == hipSuccess) e = b.alloc(n);
  };
  A(net->params, net->n_params);
  A(net->grads, net->n_params);
  A(net->m, net->n_params);
  A(net->v, net->n_params);
  A(net->act[0], B * kPix);
  for (int l = 0; l < 4; ++l) A(net->act[l + 1], B * (kConv[l].H / kConv[l].s) * (kConv[l].W / kConv[l].s) * kConv[l].co);
  A(net->dcol, colmax);
  A(net->dact, actmax);
  A(net->dact2, actmax);
  A(net->h, B * kFcHid);
  A(net->dh, B * kFcHid);
  A(net->out, B * kOut);
  A(net->dout, B * kOut);
  A(net->partial, 64);
  A(net->target, B * kOut);
  A(net->split, kSplitCap);
  A(net->colpart, (size_t)kColParts * kOut);
  if (e == hipSuccess) e = net->cells.alloc(B * kPix);
  if (e != hipSuccess) {
    delete net;
    return set_error(MVPB_E_NOMEM, "surrogate buffers: %s", hipGetErrorString(e));
  }
  // He-uniform weights (counter-based generator), zero biases and moments
  for (int t = 0; t < 12; ++t) {
    const int n = (t + 1 < 12 ? net->off[t + 1] : net->n_params) - net->off[t];
    if (t % 2 == 1) {
      e = hipMemsetAsync(net->params.p + net->off[t], 0, sizeof(float) * n, net->st);
    } else {
      const int fan_in = t < 8 ? 9 * kConv[t / 2].ci : (t == 8 ? kFcIn : kFcHid);
      hipLaunchKernelGGL(init_uniform, dim3((n + 255) / 256), dim3(256), 0, net->st, net->params.p + net->off[t], n,
                         sqrtf(6.f / fan_in), (unsigned long long)seed, (unsigned long long)net->off[t]);
    }
  }
  if (e == hipSuccess) e = hipMemsetAsync(net->m.p, 0, sizeof(float) * net->n_params, net->st);
  if (e == hipSuccess) e = hipMemsetAsync(net->v.p, 0, sizeof(float) * net->n_params, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) {
    delete net;
    return set_error(MVPB_E_DEVICE, "surrogate init: %s", hipGetErrorString(e));
  }
  ctx_retain(ctx);
  *out = net;
  return MVPB_OK;
}

extern "C" int mvpb_sur_destroy(mvpb_sur net) {
  if (!net) return MVPB_OK;
  mvpb_ctx ctx = net->ctx;
  (void)hipSetDevice(ctx_device(ctx));
  (void)hipStreamSynchronize(net->st);
  delete net;
  ctx_release_child(ctx);
  return MVPB_OK;
}

extern "C" int mvpb_sur_n_params(mvpb_sur net, int *n) {
  if (!net || !n) return set_error(MVPB_E_INVALID, "NULL argument");
  *n = net->n_params;
  return MVPB_OK;
}

extern "C" int mvpb_sur_get_params(mvpb_sur net, float *host) {
  if (!net || !host) return set_error(MVPB_E_INVALID, "NULL argument");
  (void)hipSetDevice(ctx_device(net->ctx));
  hipError_t e = hipMemcpyAsync(host, net->params.p, sizeof(float) * net->n_params, hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "get params: %s", hipGetErrorString(e));
  return MVPB_OK;
}

extern "C" int mvpb_sur_set_params(mvpb_sur net, const float *host) {
  if (!net || !host) return set_error(MVPB_E_INVALID, "NULL argument");
  for (int i = 0; i < net->n_params; ++i)
    if (!isfinite(host[i])) return set_error(MVPB_E_INVALID, "non-finite parameter %d", i);
  (void)hipSetDevice(ctx_device(net->ctx));
  hipError_t e = hipMemcpyAsync(net->params.p, host, sizeof(float) * net->n_params, hipMemcpyHostToDevice, net->st);
  if (e == hipSuccess) e = hipMemsetAsync(net->m.p, 0, sizeof(float) * net->n_params, net->st);
  if (e == hipSuccess) e = hipMemsetAsync(net->v.p, 0, sizeof(float) * net->n_params, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "set params: %s", hipGetErrorString(e));
  net->step = 0;
  return MVPB_OK;
}

static int check_batch(mvpb_sur net, int B, const void *cells) {
  if (!net || !cells) return set_error(MVPB_E_INVALID, "NULL argument");
  if (B < 1 || B > net->max_batch) return set_error(MVPB_E_INVALID, "batch %d outside [1, %d]", B, net->max_batch);
  return MVPB_OK;
}

extern "C" int mvpb_sur_infer(mvpb_sur net, int batch, const uint8_t *cells, float *out, unsigned flags) {
  int rc = check_batch(net, batch, cells);
  if (rc) return rc;
  if (!out) return set_error(MVPB_E_INVALID, "NULL output");
  (void)hipSetDevice(ctx_device(net->ctx));
  rc = stage_inputs(net, batch, cells, nullptr, flags, nullptr);
  if (!rc) rc = sur_forward(net, batch);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(out, net->out.p, sizeof(float) * batch * kOut,
                                (flags & MVPB_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess && !(flags & MVPB_F_ASYNC)) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "infer: %s", hipGetErrorString(e));
  return MVPB_OK;
}

extern "C" int mvpb_sur_gradients(mvpb_sur net, int batch, const uint8_t *cells, const float *target, float *loss,
                                  float *grads, unsigned flags) {
  int rc = check_batch(net, batch, cells);
  if (rc) return rc;
  if (!target || !grads) return set_error(MVPB_E_INVALID, "NULL argument");
  (void)hipSetDevice(ctx_device(net->ctx));
  const float *tgt = nullptr;
  rc = stage_inputs(net, batch, cells, target, flags, &tgt);
  if (!rc) rc = sur_forward(net, batch);
  if (!rc) rc = loss_and_grad_out(net, batch, tgt, loss);
  if (!rc) rc = sur_backward(net, batch);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(grads, net->grads.p, sizeof(float) * net->n_params,
                                (flags & MVPB_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "gradients: %s", hipGetErrorString(e));
  return MVPB_OK;
}

extern "C" int mvpb_sur_train_step(mvpb_sur net, int batch, const uint8_t *cells, const float *target, float lr,
                                   float *loss, unsigned flags) {
  int rc = check_batch(net, batch, cells);
  if (rc) return rc;
  if (!target) return set_error(MVPB_E_INVALID, "NULL target");
  if (!(lr > 0.f) || !isfinite(lr)) return set_error(MVPB_E_INVALID, "learning rate must be positive");
  (void)hipSetDevice(ctx_device(net->ctx));
  const float *tgt = nullptr;
  rc = stage_inputs(net, batch, cells, target, flags, &tgt);
  if (!rc) rc = sur_forward(net, batch);
  if (!rc) rc = loss_and_grad_out(net, batch, tgt, loss);
  if (!rc) rc = sur_backward(net, batch);
  if (rc) return rc;
  net->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)net->step), c2 = 1.f - powf(b2, (float)net->step);
  hipLaunchKernelGGL(adam_step, dim3((net->n_params + 255) / 256), dim3(256), 0, net->st, net->params.p, net->grads.p,
                     net->m.p, net->v.p, net->n_params, lr, b1, b2, 1e-8f, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "adam: %s", hipGetErrorString(e));
  return MVPB_OK;
}

// ---------------------------------------------------------------------------
// Checkpoints: header, then the parameters and both Adam moments (FP32,
// little-endian as in memory).
// ---------------------------------------------------------------------------
namespace {
struct SurHeader {
  char magic[8];          // "MVPBSUR1"
  int32_t version;        // 1
  int32_t n_params;
  int32_t precision;      // 0 FP32, 1 BF16 products
  int32_t reserved;
  int64_t step;           // Adam steps taken (bias-correction counter)
  uint64_t seed;          // initialisation seed of the network
};
const char kSurMagic[8] = {'M', 'V', 'P', 'B', 'S', 'U', 'R', '1'};
}  // namespace

extern "C" int mvpb_sur_save(mvpb_sur net, const char *path) {
  if (!net || !path) return set_error(MVPB_E_INVALID, "NULL argument");
  (void)hipSetDevice(ctx_device(net->ctx));
  const size_t n = (size_t)net->n_params;
  std::vector<float> buf(3 * n);
  hipError_t e = hipMemcpyAsync(buf.data(), net->params.p, sizeof(float) * n, hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess) e = hipMemcpyAsync(buf.data() + n, net->m.p, sizeof(float) * n, hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(buf.data() + 2 * n, net->v.p, sizeof(float) * n, hipMemcpyDeviceToHost, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) return set_error(MVPB_E_DEVICE, "save: %s", hipGetErrorString(e));
  SurHeader h{};
  memcpy(h.magic, kSurMagic, 8);
  h.version = 1;
  h.n_params = net->n_params;
  h.precision = net->bf16 ? 1 : 0;
  h.step = net->step;
  h.seed = net->seed;
  FILE *f = fopen(path, "wb");
  if (!f) return set_error(MVPB_E_INVALID, "cannot open %s for writing", path);
  const bool ok = fwrite(&h, sizeof h, 1, f) == 1 && fwrite(buf.data(), sizeof(float), 3 * n, f) == 3 * n;
  const bool closed = fclose(f) == 0;
  if (!ok || !closed) return set_error(MVPB_E_INVALID, "write to %s failed", path);
  return MVPB_OK;
}

extern "C" int mvpb_sur_load(mvpb_ctx ctx, const char *path, int max_batch, mvpb_sur *out) {
  if (!ctx || !path || !out) return set_error(MVPB_E_INVALID, "NULL argument");
  FILE *f = fopen(path, "rb");
  if (!f) return set_error(MVPB_E_INVALID, "cannot open %s", path);
  SurHeader h{};
  std::vector<float> buf;
  bool ok = fread(&h, sizeof h, 1, f) == 1 && memcmp(h.magic, kSurMagic, 8) == 0 && h.version == 1 &&
            (h.precision == 0 || h.precision == 1) && h.step >= 0;
  int off[12];
  ok = ok && h.n_params == param_offsets(off);
  if (ok) {
    buf.resize(3 * (size_t)h.n_params);
    ok = fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;   // nothing after the moments
  }
  fclose(f);
  if (!ok) return set_error(MVPB_E_INVALID, "%s is not a surrogate checkpoint of this network", path);
  for (float x : buf)
    if (!isfinite(x)) return set_error(MVPB_E_INVALID, "%s holds non-finite values", path);
  mvpb_sur net = nullptr;
  int rc = mvpb_sur_create(ctx, max_batch, h.precision, h.seed, &net);
  if (rc) return rc;
  const size_t n = (size_t)h.n_params;
  hipError_t e = hipMemcpyAsync(net->params.p, buf.data(), sizeof(float) * n, hipMemcpyHostToDevice, net->st);
  if (e == hipSuccess) e = hipMemcpyAsync(net->m.p, buf.data() + n, sizeof(float) * n, hipMemcpyHostToDevice, net->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(net->v.p, buf.data() + 2 * n, sizeof(float) * n, hipMemcpyHostToDevice, net->st);
  if (e == hipSuccess) e = hipStreamSynchronize(net->st);
  if (e != hipSuccess) {
    mvpb_sur_destroy(net);
    return set_error(MVPB_E_DEVICE, "load: %s", hipGetErrorString(e));
  }
  net->step = h.step;
  *out = net;
  return MVPB_OK;
}
