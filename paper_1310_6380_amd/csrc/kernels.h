// Device work descriptors and kernel launchers of the mvpb library.
#pragma once

#include "common.h"

typedef struct mvpb_ctx_s *mvpb_ctx;

namespace mvpb {

// Error reporting and context access shared by the translation units of the
// library (defined with the C-ABI entry points).
int set_error(int code, const char *fmt, ...);
hipStream_t ctx_stream(mvpb_ctx c);
int ctx_device(mvpb_ctx c);
bool ctx_closing(mvpb_ctx c);
void ctx_retain(mvpb_ctx c);         // a child object (cell, plan, network) now holds the context
void ctx_release_child(mvpb_ctx c);  // ... and lets it go

// Largest reduced-operator order handled by the eigensolver kernels
// (2N <= MAX_N; vectors of this length are staged in LDS).
constexpr int MAX_N = 4096;
// Half bandwidth of the band form produced by the first reduction stage
// (also the length of the bulge-chasing reflectors of the second stage).
constexpr int HB = 16;
// Columns of zeros after the n columns of the bulge-chasing band copy: every
// entry a block reads past row or column n - 1 is then a stored zero, and the
// block loads need no bounds masks.
constexpr int WB_PAD_COLS = HB;
// LDS budget of the back-transform's eigenvector block.
constexpr int BT_LDS_BYTES = 128 * 1024;
// Most bands of a solve that ends with the FP64 Rayleigh-Ritz step (its
// block is held in LDS; the FP32 reduction always needs that step).
constexpr int RR_MAX_BANDS = 64;
// Most bands of an FP64 solve: beyond RR_MAX_BANDS the frequencies and
// vectors come straight from the tridiagonal eigenpairs and the
// back-transform (the FP64 reduction is backward stable; the refinement is
// for the FP32 one).
constexpr int MAX_BANDS = 256;

// One (cell, k) work item of the eigensolve.  All pointers are device memory
// owned by the solve that built the item table.  Buffers marked (R) hold
// complex numbers of the reduction precision: complex double on the FP64
// path, complex float on the FP32 one.
struct EigItem {
  // operator formation
  const cd *coef;   // coefficient matrices of C(k) (plan-owned): dim 0: 15 of N x N (isotropic
                    // planar layout); dim 2, 3: (dim+1)(dim+2)/2 of n x n (general layout)
  double kap1, kap2, kap3;  // Cartesian Bloch vector kappa = 2 pi T Q
  int N;            // plane waves
  int n;            // order of the operator (2N planar, 3N spatial)
  int dim;          // coefficient layout, see coef
  int nb;           // bands wanted
  int slot;         // row of this item's frequencies in the output
  // stage 1: dense -> band
  void *A;          // (R) n x n working matrix; the panels' reflectors stay below the band
  cd *Ak;           // n x n kept copy of C(k) for Rayleigh-Ritz (always FP64)
  void *X0;         // (R) n x HB product of the trailing matrix with the panel reflectors
  void *Wm;         // (R) n x HB rank-2HB update factor
  void *M0p;        // (R) ceil(n/64) x HB x HB Gram partials
  void *T1;         // (R) ceil(n/HB) x HB x HB compact-WY factors of the panels
  // stage 2: band -> tridiagonal
  void *WB;         // (R) n x (2 HB + 1) band working copy
  void *V2;         // (R) reflectors of the bulge chasing, HB entries each; per sweep in chunks of 8 blocks, entry-major in a chunk
  void *tau2;       // (R) their scalars
  double *d;        // n diagonal
  double *e;        // n off-diagonal (real)
  int *flag;        // n + 2: [0] nonzero if the bulge chasing gave up (its frequencies are then NaN),
                    // [1] abort, [2 + i] progress of sweep i
  // tridiagonal eigenproblem
  double *X;        // n x nb eigenvectors of the tridiagonal matrix (row-major)
  double *lu;       // 5 n x nb factorisation scratch (orders above the LDS limit)
  double *lam_t;    // nb eigenvalues of the tridiagonal matrix
  // back-transform and refinement
  cd *Y;            // n x nb eigenvectors of C(k) (FP64, input of Rayleigh-Ritz)
  void *Yb;         // (R) back-transform output (== Y on the FP64 path)
  cd *Z;            // n x nb: C Y, then the refined eigenvectors
  cd *Gp;           // ceil(n/64) x 2 x nb x nb Gram partials of Rayleigh-Ritz
  cd *Lr;           // nb x nb Cholesky factor of Y^H Y
  double *lam;      // nb refined eigenvalues (lambda = omega^2)
  double *omega;    // nb output frequencies (device)
  double *acc;      // 1: largest a posteriori relative frequency error estimate of the refined bands
  int check;        // 1: compute that estimate (FP32 reduction), 0: acc = 0
};

// assembly.hip
hipError_t launch_structure_factors_f64(const int32_t *phase, const double *wtab, int nx, int ny, int M1,
                                        int M2, double area, cd *X, cd *F, hipStream_t st);
// Matrix-core variant: prec 0 = FP64, 1 = FP32, 2 = BF16 inputs (FP32 accumulate),
// 3 = split BF16 (hi + lo inputs, three BF16 products, FP32 accumulate).
// X: scratch of 8 * nx * (4 M2 + 1) doubles.
hipError_t launch_structure_factors_mfma(int prec, const int32_t *phase, const double *wtab, int nx, int ny, int M1,
                                         int M2, double area, double *X, cd *F, hipStream_t st);
// Polygon cells: edges[e] = {mid_x, mid_y, d_x, d_y} (Cartesian, d = end -
// start in the polygon's orientation), ephase[e] its polygon's phase;
// f0[4] = the weighted phase areas (the dG = 0 entry).  X: scratch of
// sf_poly_scratch_bytes(n_edges, M1, M2) bytes.
size_t sf_poly_scratch_bytes(int n_edges, int M1, int M2);
// Stress modes S = -Phi^-1 H* U (isotropic cells).  stress_rhs: from U
// [n_k][nb][2N] (complex) the three right-hand sides X[t][j] (N x nb,
// column-major), j = 0: V11 + V22, 1: V11 - V22, 2: V12 with V = H* U;
// stress_combine: S[t][b][3N] from Z[t][j] = (Sigma^-1, Delta^-1, Delta^-1)
// applied to X[t][j].  Q: device [n_k][2].
hipError_t launch_stress_rhs(const cd *U, const double *Q, int n_k, int nb, int M1, int M2, const double T[4],
                             double area, cd *X, hipStream_t st);
hipError_t launch_stress_combine(const cd *Z, int n_k, int nb, int N, cd *S, hipStream_t st);
hipError_t launch_structure_factors_poly(const double *edges, const int *ephase, const double *wtab, int n_edges,
                                         const double T[4], const double f0[4], int M1, int M2, cd *X, cd *F,
                                         hipStream_t st);
// count cells: F [count][4][4M1+1][4M2+1], T [count][3][N][N] (Sigma, Delta, rho blocks)
hipError_t launch_toeplitz_scatter(const cd *F, int M1, int M2, int N, cd *T, int count, hipStream_t st);
// count pixel cells of one grid size in one launch pair: device tables of phase
// maps, weight tables and areas; X: count * 8 nx (4M2+1) doubles; F: count * 4 (4M1+1)(4M2+1).
hipError_t launch_structure_factors_mfma_batch(int prec, const int32_t *const *phases, const double *const *wtabs,
                                               const double *areas, int count, int nx, int ny, int M1, int M2,
                                               double *X, cd *F, hipStream_t st);
hipError_t launch_combine(const cd *Xp, int N, double s, cd *coef, hipStream_t st);
// count cells: products Xp + c 18 N^2, coefficients coef + c 15 N^2, scale scales[c] (device)
hipError_t launch_combine_batch(const cd *Xp, int N, const double *scales, cd *coef, int count, hipStream_t st);
hipError_t launch_form_operator(const EigItem *items, int n_items, int n_max, bool fp32, hipStream_t st);

// general.hip: general compliance and voxel cells (full Phi).
// Weight fields [nf][4M1+1][4M2+1][4M3+1] of a pixel (nz = 1, M3 = 0) or
// voxel cell; X1: nf nx ny (4M3+1), X2: nf nx (4M2+1)(4M3+1) complex scratch.
hipError_t launch_structure_factors_general(const int32_t *phase, const double *gw, int nf, int nx, int ny, int nz,
                                            int M1, int M2, int M3, double vol, cd *X1, cd *X2, cd *F,
                                            hipStream_t st);
// out (nblk N square, column-major): block (s, t) = Toeplitz matrix of field fmap[s nblk + t].
hipError_t launch_toeplitz_blocks(const cd *F, int M1, int M2, int M3, int N, int nblk, const int *fmap, cd *out,
                                  hipStream_t st);
hipError_t launch_form_operator_general(const EigItem *items, int n_items, int n_max, bool fp32, hipStream_t st);
// X = H* U per point (U [n_k][nb][d N], X [n_k][nb][n_s N]); Q [n_k][d] device; T row-major d x d.
hipError_t launch_stress_rhs_general(const cd *U, const double *Q, int n_k, int nb, int d, int M1, int M2, int M3,
                                     const double *T, double vol, cd *X, hipStream_t st);

// sensitivity.hip: d lambda / d w_f of every pixel / voxel for n_items (point,
// band) items: U [items][d N], S [items][n_s N], omega [items] (device);
// scratch Cw: items nf (4M1+1)(4M2+1)(4M3+1), Y1: items nf nx (4M2+1)(4M3+1),
// Y2: items nf nx ny (4M3+1) complex; G [items][nf][nx][ny][nz].
hipError_t launch_sensitivities(const cd *U, const cd *S, const double *omega, int n_items, int d, int M1, int M2,
                                int M3, int nx, int ny, int nz, double vol, cd *Cw, cd *Y1, cd *Y2, double *G,
                                hipStream_t st);

// dense.hip
// Cholesky (lower, in place) and explicit inverse of the factor for `count`
// matrices A[b] (N x N, column-major); Linv[b] receives L^-1 (lower, the
// strict upper part zeroed).  status[b] = 0 on success, j+1 if the pivot of
// column j was not positive.
hipError_t launch_potrf_trtri(cd *const *A, cd *const *Linv, int *status, int count, int N, hipStream_t st);
hipError_t launch_identity_if_failed(cd *const *Linv, const int *status, int count, int N, hipStream_t st);

enum Op { OP_N = 0, OP_C = 1 };
// Batched complex GEMM: C[b] = alpha * op(A[b]) * diag(s[b]) * op(B[b]) + beta * C[b].
// All matrices column-major; s[b] may be NULL (no scaling); M x K by K x N.
struct GemmBatch {
  const cd *const *A;
  const cd *const *B;
  cd *const *C;
  const double *const *s;
  int lda, ldb, ldc;
};
hipError_t launch_zgemm(Op opA, Op opB, int M, int N, int K, cd alpha, GemmBatch bt, cd beta, int count,
                        hipStream_t st);

// band.hip
hipError_t init_band_attributes();
// Stage 1 (dense -> band) and stage 2 (band -> tridiagonal d, e) for every item.
// A set of items (consecutive in the device item table) with its size range
// and the stream its launches go to.
struct ItemPart {
  const EigItem *items = nullptr;
  int n_items = 0, n_min = 0, n_max = 0;
  hipStream_t stream = nullptr;
  // look-ahead: the trailing update of panel p runs on `aside` while panel
  // p+1 is factored on `stream`; ev holds 2 stage1_steps(n_max) events
  // (W of panel p formed, update of panel p done), each recorded once
  hipStream_t aside = nullptr;
  const hipEvent_t *ev = nullptr;
};
// Panels of stage 1 for an operator of order n (those with rows below the band).
inline int stage1_steps(int n) { return n > HB ? (n - HB - 1) / HB + 1 : 0; }
// Reduction to band form (stage 1) of every part, the parts' launches
// interleaved step by step on their own streams; every part's `stream` has
// waited for its `aside` stream when the call returns.
hipError_t launch_stage1(const ItemPart *parts, int n_parts, bool fp32);
// Band to tridiagonal (stage 2, bulge chasing) and d, e of all items; ctl
// points to hb2st_ctl_ints(n_items) ints of device memory.  Launch shape:
// group = consecutive sweeps dealt to one workgroup's wavefronts (a divisor
// of 8; 0: 8), wg_max = most workgroups per item (0: 4; fewer when the
// launch would not be resident at once), spin_limit = polls of a bounded
// hand-over wait before the item gives up (0: 2^24).
struct Stage2Shape {
  int group = 0;
  int wg_max = 0;
  long long spin_limit = 0;
};
size_t hb2st_ctl_ints(int n_items);
hipError_t launch_stage2(const EigItem *items, int n_items, int n_max, bool fp32, int *ctl, const Stage2Shape &sh,
                         hipStream_t st);
// Eigenvectors of C(k) from those of the tridiagonal matrix (X -> Y).
hipError_t launch_backtransform(const EigItem *items, int n_items, int n_min, int n_max, int nb, bool fp32,
                                hipStream_t st);
int backtransform_cols(int n_max, bool fp32);
long long refl_total(int n);   // number of stage-2 reflectors of an item of order n

// eigen.hip
hipError_t init_kernel_attributes();  // once per device, before the first launch
// side: a stream (with two events) on which the inverse iteration of cluster
// members runs beside the twisted factorizations of the isolated eigenvalues
// (they write disjoint eigenvector columns), or nullptr for one stream.
hipError_t launch_tridiag_eig(const EigItem *items, int n_items, int n_max, int nb, hipStream_t st,
                              hipStream_t side = nullptr, hipEvent_t ev_fork = nullptr, hipEvent_t ev_join = nullptr);
hipError_t launch_rayleigh_ritz(const EigItem *items, int n_items, int n_max, int nb, bool check, hipStream_t st);
// Solves beyond RR_MAX_BANDS (FP64): lambda, omega from the tridiagonal
// eigenvalues, no estimate (acc = 0); the vectors stay in Y.
hipError_t launch_tridiag_results(const EigItem *items, int n_items, int nb, hipStream_t st);

}  // namespace mvpb
