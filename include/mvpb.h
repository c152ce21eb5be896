/*
 * mvpb -- mixed-variational phononic band structures on one MI355X (gfx950).
 *
 * C-ABI of the library.  Plain pointers and sizes only.  The method is the
 * mixed-variational (Nemat-Nasser / Srivastava) Galerkin formulation of
 * arXiv:1310.6380:
 *   - unit cell, lattice vectors h^1, h^2 and Bloch vector k = Q_i q^i: Sec. 2;
 *   - Bloch-Fourier basis with cutoff M1, M2 (alpha in [-M1,M1], beta in
 *     [-M2,M2]): Sec. 2.3 and eq. (approximation2d);
 *   - matrices H, Omega, Phi, H* = -H^T: Sec. 4.1, eqs. (eh), (eo), (ep);
 *   - eigenproblem (H Phi^-1 H*) U = lambda Omega U, omega = sqrt(lambda):
 *     Sec. 3, eq. (eigenvalueproblem), solved in generalized Hermitian form.
 *
 * Conventions
 *   Units: SI (lattice in metres, E in Pa, rho in kg/m^3, omega in rad/s).
 *   Status: every call returns an int status (MVPB_OK = 0 or a negative
 *     MVPB_E_* code).  On error out-parameters are left untouched and a
 *     message is available from mvpb_last_error() on the calling thread.
 *     The library never aborts or exits.
 *   Ownership: all arrays are owned by the caller.  *_create calls deep-copy
 *     their inputs, so the caller may free them on return.  Handles are owned
 *     by the library and released only by the matching *_destroy.  A
 *     context destroyed while cells or plans of it are alive stays usable by
 *     them and is freed together with the last one; it accepts no new work.
 *   Streams: all device work of a context runs on the stream given to
 *     mvpb_ctx_create (NULL = a stream owned by the context).  Calls return
 *     after the stream has finished unless MVPB_F_ASYNC is passed (then
 *     device outputs are valid once the stream has drained, and device
 *     errors surface at the next synchronising call).
 *   Threads: a context and its cells/plans must not be used from two host
 *     threads at once.
 */
#ifndef MVPB_H
#define MVPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mvpb_ctx_s *mvpb_ctx;
typedef struct mvpb_cell_s *mvpb_cell;
typedef struct mvpb_plan_s *mvpb_plan;

enum {
  MVPB_OK = 0,
  MVPB_E_INVALID = -1,     /* bad argument (NULL, size, NaN, property range ...) */
  MVPB_E_NOT_PD = -2,      /* a compliance/density matrix is not positive definite */
  MVPB_E_NOMEM = -3,       /* device allocation failed or workspace cap exceeded */
  MVPB_E_DEVICE = -4,      /* HIP runtime error */
  MVPB_E_UNSUPPORTED = -5, /* valid request that the library does not implement */
  MVPB_E_ACCURACY = -6     /* a solve with the FP32 reduction (MVPB_PREC_EIG_FP32_RR64)
                              estimates a frequency error above the context's bar (see
                              mvpb_ctx_set_accuracy); unlike every other error, the
                              outputs of that solve ARE written */
};

/* Property table layouts (one row per phase). */
enum {
  MVPB_PROP_ISO_E_NU_RHO = 0, /* E [Pa], nu, rho [kg/m^3]; isotropic (planar cells: plane
                                 strain, Sec. 4) */
  MVPB_PROP_VOIGT_D_RHO = 1   /* general compliance: the engineering-Voigt compliance matrix
                                 d (strain = d stress with engineering shear strains, i.e. the
                                 weights c_s c_t D_jkmn of the Phi blocks of Sec. 4.1 eq. (ep),
                                 c = 1 on normal and 2 on shear components: d13 = 2 D1112,
                                 d33 = 4 D1212 in the plane), upper triangle row by row, then
                                 rho [kg/m^3].  Planar cells (stress order 11, 22, 12): d11,
                                 d12, d13, d22, d23, d33, rho (7 values); voxel cells (11, 22,
                                 33, 23, 13, 12): the 21 entries d11 .. d16, d22 .. d26, ...,
                                 d66, then rho (22 values).  Positive definite, rho > 0.
                                 Pixel and voxel cells only. */
};

/* Precision of a plan: bit flags.  The structure-factor contraction runs on
 * the matrix cores (FP64 by default); the low two bits select one of FP64,
 * SF_FP32, SF_BF16 and SF_BF16X3.  EIG_FP32_RR64 may be combined with any. */
enum {
  MVPB_PREC_FP64 = 0,           /* everything in FP64 */
  MVPB_PREC_SF_FP32 = 1,        /* structure factors: FP32 inputs, FP32 accumulate */
  MVPB_PREC_SF_BF16 = 2,        /* structure factors: BF16 inputs, FP32 accumulate */
  MVPB_PREC_SF_BF16X3 = 3,      /* structure factors: every input split into two BF16
                                   parts hi + lo, each product as the three BF16 products
                                   lo*hi + hi*lo + hi*hi, FP32 accumulate (Henry, Tang and
                                   Heinecke, ARITH 2019) */
  MVPB_PREC_EIG_FP32_RR64 = 4,  /* FP32 reduction to tridiagonal form and back-transform,
                                   FP64 Rayleigh-Ritz refinement on the FP64 operator */
  MVPB_PREC_SF_PLAIN64 = 8,     /* structure factors by the scalar FP64 kernel (cross-check) */
  MVPB_PREC_GENERAL = 16        /* build an isotropic planar cell's plan in the general layout
                                   (full Phi, as for MVPB_PROP_VOIGT_D_RHO cells; cross-check) */
};

/* Flags of mvpb_solve / mvpb_solve_batch. */
enum {
  MVPB_F_DEVICE_PTRS = 1, /* omega / U are device pointers (else host pointers) */
  MVPB_F_ASYNC = 2        /* do not wait for the stream before returning */
};

/* Last error message of the calling thread (valid until its next mvpb call). */
const char *mvpb_last_error(void);

/* Library version string. */
const char *mvpb_version(void);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (NULL: the context creates its own).  `workspace_cap` bounds the bytes of
 * device workspace a single solve may allocate (0 = no bound); a solve that
 * needs more returns MVPB_E_NOMEM. */
int mvpb_ctx_create(int device, void *hip_stream, size_t workspace_cap, mvpb_ctx *out);
int mvpb_ctx_destroy(mvpb_ctx ctx);

/* Accuracy bar of the mixed-precision eigensolve.  After the FP64
 * Rayleigh-Ritz step of a solve with the FP32 reduction, every refined pair
 * (theta, z) has its residual r = C z - theta z computed in FP64 on the FP64
 * operator, and the error of theta is estimated to second order as
 * |r|^2 / (rho - theta) with rho = r^H C r / |r|^2 the Rayleigh quotient of
 * the residual (r is orthogonal to the Ritz space, so rho - theta is its
 * effective distance to the rest of the spectrum; |r| if rho <= theta),
 * expressed as a relative frequency error: estimate / (2 theta), or
 * estimate / (2 theta_top) for bands below 1e-3 of the top frequency
 * (acoustic modes at and next to Gamma).  It is an estimate, not a bound.
 * A synchronous mvpb_solve / mvpb_solve_batch with the FP32 reduction
 * returns MVPB_E_ACCURACY (outputs written) when the largest estimate
 * exceeds `tol` (default 1e-5; 0 turns the check off).  FP64 solves report
 * 0 and are never refused.  With MVPB_F_ASYNC nothing is checked. */
int mvpb_ctx_set_accuracy(mvpb_ctx ctx, double tol);
/* Largest estimate of the last synchronous solve on ctx (0 before any). */
int mvpb_ctx_last_accuracy(mvpb_ctx ctx, double *estimate);

/* A unit cell given as an nx x ny pixel map of phase ids.
 * lattice[4] = {h1x, h1y, h2x, h2y} (rows of the matrix A of Sec. 4).
 * phase[i*ny + j] is the phase of pixel (i, j), i along h1, in [0, n_phases).
 * Pixel (i,j) covers fractional coordinates H1 in [i/nx,(i+1)/nx],
 * H2 in [j/ny,(j+1)/ny].  props: n_phases rows in the layout prop_kind
 * (ISO: E > 0, -1 < nu < 0.5, rho > 0).  Phases with no pixel are allowed.
 * Host pointers; deep-copied. */
int mvpb_cell_create_pixels(mvpb_ctx ctx, const double lattice[4], int nx, int ny,
                            const int32_t *phase, int n_phases, int prop_kind,
                            const double *props, mvpb_cell *out);
/* A three-dimensional unit cell (the spatial form of the method: Sec. 2,
 * Sec. 2.3 with test functions in three fractional coordinates,
 * 3(2M+1)^3 displacement and 6(2M+1)^3 stress unknowns) given as an
 * nx x ny x nz voxel map.  lattice[9] = rows h1, h2, h3 of A.
 * phase[(i*ny + j)*nz + k] is the phase of voxel (i, j, k), i along h1, k
 * along h3; voxel (i,j,k) covers H1 in [i/nx,(i+1)/nx], H2 in [j/ny,(j+1)/ny],
 * H3 in [k/nz,(k+1)/nz].  props: n_phases rows of kind ISO (E, nu, rho;
 * three-dimensional isotropic compliance) or VOIGT_D_RHO (22 values).
 * Plans of voxel cells come from mvpb_plan_create3 and use the general
 * layout.  Host pointers; deep-copied. */
int mvpb_cell_create_voxels(mvpb_ctx ctx, const double lattice[9], int nx, int ny, int nz,
                            const int32_t *phase, int n_phases, int prop_kind,
                            const double *props, mvpb_cell *out);
/* A unit cell given as polygons (Sec. 4.1: the subdomain integrals of
 * eqs. (eo), (ep) taken exactly over each polygon instead of the centroid
 * rule of Sec. 3; polygons may carry any number of phases, as in the
 * hexagonal examples of Sec. 5).  Polygon i has phase poly_phase[i] and the
 * vertices xy[2v], xy[2v+1] (Cartesian, same units as the lattice) for v in
 * [vert_offset[i], vert_offset[i+1]); vert_offset[0] = 0, at least 3
 * vertices each, the closing edge implied.  A counter-clockwise polygon adds
 * its area to its phase, a clockwise one subtracts it (a hole is a clockwise
 * copy of its boundary in the enclosing phase).  The signed areas must tile
 * the cell: their sum equals |det A| to 1e-9 relative and no phase ends up
 * negative, else MVPB_E_INVALID.  props of kind ISO only.  Structure
 * factors of polygon cells are computed in FP64 for every precision setting.
 * Host pointers; deep-copied. */
int mvpb_cell_create_polygons(mvpb_ctx ctx, const double lattice[4], int n_polys,
                              const int32_t *poly_phase, const int32_t *vert_offset,
                              const double *xy, int n_phases, int prop_kind,
                              const double *props, mvpb_cell *out);
int mvpb_cell_destroy(mvpb_cell cell);

/* Build the k-independent part of the method for cutoff (M1, M2):
 * structure factors of every phase on the (4M1+1)x(4M2+1) difference grid,
 * the compliance matrix Phi and density matrix Omega (Sec. 4.1 eqs. (eo),
 * (ep)), their Cholesky factors, and the coefficient matrices of the
 * reduced operator, which is quadratic in the Bloch vector.  M1, M2 >= 0,
 * N = (2M1+1)(2M2+1) <= 4096.  Returns MVPB_E_NOT_PD if Phi or Omega is
 * not positive definite. */
int mvpb_plan_create(mvpb_cell cell, int M1, int M2, int precision, mvpb_plan *out);
/* Plans of the general layout: used for cells whose compliance is given as
 * a full matrix (MVPB_PROP_VOIGT_D_RHO), for voxel cells, and on request
 * (MVPB_PREC_GENERAL).  The whole stress-space compliance matrix Phi
 * (n_s = 3N or 6N square, Sec. 4.1 eq. (ep) and its spatial form) and
 * Omega are factored; the reduced operator is quadratic in the Bloch vector
 * with (d+1)(d+2)/2 coefficient matrices of order n_u = dN (d = 2 planar,
 * 3 spatial).  Structure factors are computed in FP64 for every precision
 * setting; MVPB_PREC_EIG_FP32_RR64 applies.  Requires d N <= 4096.
 * mvpb_plan_create3 takes the cutoff of every axis (M3 = 0 for a planar
 * cell, which is then the same as mvpb_plan_create). */
int mvpb_plan_create3(mvpb_cell cell, int M1, int M2, int M3, int precision, mvpb_plan *out);
/* Plans for n cells of one context at once (same precision): cells with
 * equal cutoffs share batched launches for the factorisations and the
 * coefficient GEMMs.  out[i] receives the plan of cells[i]; on error no plan
 * is returned (MVPB_E_NOT_PD names the failing cell index). */
int mvpb_plan_create_batch(mvpb_ctx ctx, int n, const mvpb_cell *cells, const int *M1, const int *M2,
                           int precision, mvpb_plan *out);
/* n_u = dN displacement unknowns, n_s = 3N (planar) or 6N (spatial) stress
 * unknowns (Sec. 4.1; Sec. 2.3). */
int mvpb_plan_dofs(mvpb_plan plan, int *n_u, int *n_s);
int mvpb_plan_destroy(mvpb_plan plan);

/* Solve for the lowest n_bands at each of n_k Bloch vectors.
 * Q[d*t + i] = Q_i of point t (k = Q_i q^i, finite), d = 2 for planar cells
 * and 3 for voxel cells.
 * omega[t*n_bands + b]: frequencies in rad/s, ascending per point
 *   (sqrt(max(lambda, 0))).
 * U: NULL or space for n_k*n_bands*n_u complex values (interleaved re, im),
 *   U[((t*n_bands + b)*n_u + c*N + r)], the coefficients of displacement
 *   component c in the plane-wave order I = (alpha+M1)(2M2+1)+(beta+M2)
 *   (voxel cells: I = ((alpha+M1)(2M2+1)+(beta+M2))(2M3+1)+(gamma+M3));
 *   normalised to U^H Omega U = 1 with the largest-modulus entry real > 0.
 * 1 <= n_bands <= min(n_u, 256) for FP64 plans: up to 64 bands the
 * frequencies and vectors are refined by an FP64 Rayleigh-Ritz step (its
 * block is held in on-chip memory), beyond that they come straight from
 * the FP64 tridiagonal eigenpairs and the back-transform.  Plans with
 * MVPB_PREC_EIG_FP32_RR64 take 1 <= n_bands <= min(n_u, 64).  Q, omega and
 * U are host pointers unless MVPB_F_DEVICE_PTRS is set (then omega and U
 * are device pointers; Q stays on the host).  If the device could not finish a point (the reduction to
 * tridiagonal form gave up waiting on a hand-over), its frequencies are NaN;
 * with host pointers the call then returns MVPB_E_DEVICE. */
int mvpb_solve(mvpb_plan plan, int n_k, const double *Q, int n_bands, double *omega, double *U,
               unsigned flags);

/* Stress modes S = -Phi^-1 H* U (Sec. 3, after eq. (eigenvalueproblem); H
 * and Phi of Sec. 4.1 eqs. (eh), (ep)) of displacement modes U, for every
 * plan (isotropic and general layouts).  Q as for mvpb_solve; U:
 * n_k*n_bands*n_u complex values in the layout mvpb_solve writes (any
 * normalisation: S is linear in U).  S: space for n_k*n_bands*n_s complex
 * values, S[((t*n_bands + b)*n_s + c*N + r)], c the Voigt stress component
 * (planar 11, 22, 12; spatial 11, 22, 33, 23, 13, 12), plane-wave order as
 * for U.  Host pointers unless MVPB_F_DEVICE_PTRS (then U and S are device
 * pointers).  1 <= n_bands <= n_u. */
int mvpb_stress_modes(mvpb_plan plan, int n_k, const double *Q, int n_bands, const double *U,
                      double *S, unsigned flags);

/* Sensitivities of the eigenvalues lambda = omega^2 to the material of every
 * pixel or voxel, for gradient-based band-structure design (Sec. 1 and
 * Sec. 6 motivate optimisation).  Differentiating eq. (eigenvalueproblem)
 * (A U = lambda Omega U, A = H Phi^-1 H*, Sec. 3) at a simple eigenvalue
 * with U^H Omega U = 1 gives d lambda = -S^H dPhi S - lambda U^H dOmega U,
 * S = -Phi^-1 H* U.  The design variables of element p are its weight fields
 * w_f: the engineering-Voigt compliance entries (the Phi weights of Sec. 4.1
 * eq. (ep); upper triangle row by row, a shear-normal entry w_st moving
 * both blocks (s, t) and (t, s)) and, last, its density (eq. (eo)):
 * 7 fields for planar cells, 22 for voxel cells.
 * Q, n_bands as for mvpb_solve; omega [n_k][n_bands] and U
 * [n_k][n_bands][n_u] as mvpb_solve returned them (U normalised to
 * U^H Omega U = 1).  G: space for n_k*n_bands*nf*cells doubles,
 * G[((t*n_bands + b)*nf + f)*cells + (i*ny + j)*nz + k] = d lambda_b(k_t) /
 * d w_f(i, j, k) (nz = 1 for pixel cells).  At a degenerate eigenvalue only
 * the sum over the degenerate bands is defined.  Pixel and voxel cells
 * only (MVPB_E_UNSUPPORTED for polygon cells).  Host pointers unless
 * MVPB_F_DEVICE_PTRS (then omega, U and G are device pointers; Q stays on
 * the host). */
int mvpb_band_sensitivities(mvpb_plan plan, int n_k, const double *Q, int n_bands, const double *omega,
                            const double *U, double *G, unsigned flags);

/* Many plans at once: all (plan, k) items in one batched launch sequence
 * (captured in a HIP graph and replayed).  n_k[p] points for plan p taken
 * from Q[p] (host pointers), results to omega[p][t*n_bands + b] (host
 * pointers, or device pointers with MVPB_F_DEVICE_PTRS; Q[p] holds d
 * components per point as for mvpb_solve).  Every plan must belong to ctx
 * and have n_u >= n_bands. */
int mvpb_solve_batch(mvpb_ctx ctx, int n_plans, const mvpb_plan *plans, const int *n_k,
                     const double *const *Q, int n_bands, double *const *omega, unsigned flags);

/* Band structure of many pixel cells in one call, plan build included:
 * the structure factors of every cell (Sec. 4.1, per-pixel closed forms
 * summed on the matrix cores), its Toeplitz blocks (eqs. (eh), (eo), (ep)),
 * the Cholesky factors and coefficient matrices of the reduced operator
 * C(k) (Sec. 3, eq. (eigenvalueproblem)), and the eigensolve of every
 * (cell, k) pair, enqueued as ONE captured HIP graph.  The graph is kept
 * (at most 4 per context, least recently used dropped) and replayed by a
 * later call of the same shape: the same cell count, and per cell (in
 * cutoff order) the same cutoff, pixel grid and k count, with the same
 * n_bands, precision and launch shapes.  Per-call data (phase maps, phase
 * tables, lattices, Bloch vectors) reach the kernels through device tables
 * uploaded before each launch, so a replay needs no host work beyond one
 * copy.  The plans are not kept: their matrices live in a context-owned
 * workspace (grow-only, within the context's workspace cap).
 *   cells[i]: isotropic pixel cells of ctx (MVPB_E_UNSUPPORTED for polygon,
 *             voxel and general-compliance cells);
 *   M1[i], M2[i]: cutoffs, 2 N <= the plan limit;
 *   precision: as for mvpb_plan_create without MVPB_PREC_SF_PLAIN64 and
 *             MVPB_PREC_GENERAL (MVPB_E_UNSUPPORTED);
 *   n_k[i] >= 0 points of cell i in Q[i] (host, 2 reduced coordinates
 *             each), results to omega[i][t * n_bands + b] (host pointers, or
 *             device pointers with MVPB_F_DEVICE_PTRS);
 *   n_bands: 1 .. min(2 N_i, 256), or 64 with MVPB_PREC_EIG_FP32_RR64.
 * Always returns after the results are written (MVPB_F_ASYNC is ignored).
 * Errors: MVPB_E_NOT_PD names the first cell (caller's index) whose
 * compliance or density matrix failed to factor (its results are not
 * meaningful, the other cells' are); MVPB_E_NOMEM if the workspace would
 * exceed the cap; MVPB_E_ACCURACY and MVPB_E_DEVICE as for mvpb_solve. */
int mvpb_solve_cells(mvpb_ctx ctx, int n_cells, const mvpb_cell *cells, const int *M1, const int *M2,
                     int precision, const int *n_k, const double *const *Q, int n_bands,
                     double *const *omega, unsigned flags);

/* Structure factors of the general layout (pixel and voxel cells):
 * F[((f*(4M1+1) + m+2M1)*(4M2+1) + q+2M2)*(4M3+1) + r+2M3] (complex,
 * interleaved) = sum_p w_f(p) int_{Omega_p} exp(i 2 pi (m H1 + q H2 + r H3)) dx
 * for the fields f = the upper triangle of the engineering-Voigt compliance
 * matrix (row by row) and, last, rho: 7 fields for planar cells (M3 = 0),
 * 22 for voxel cells.  FP64.  F: host pointer. */
int mvpb_structure_factors_general(mvpb_cell cell, int M1, int M2, int M3, double *F);

/* Phase-summed structure factors of a cell on the difference grid
 * (debug/parity access to the first step of the method):
 * F[(w*(4M1+1) + m+2M1)*(4M2+1) + q+2M2] (complex, interleaved) for the
 * weights w = 0: d11+d12, 1: d11-d12, 2: rho, 3: 1, where
 * F_w(m,q) = sum_p w_p int_{Omega_p} exp(i 2 pi (m H1 + q H2)) dx.
 * `precision` selects the FP64, FP32 or BF16 contraction.  F: host pointer,
 * 4*(4M1+1)*(4M2+1) complex values. */
int mvpb_structure_factors(mvpb_cell cell, int M1, int M2, int precision, double *F);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * structure factors as mvpb_structure_factors, same kernels and layout, but
 * F is a DEVICE pointer owned by the caller (4*(4M1+1)*(4M2+1) complex
 * values) and the call allocates nothing.  The two DFT passes keep their
 * intermediate sums in a fixed device array of 16 MiB per GPU (held until
 * the process ends); its address is looked up when a context is created on
 * the device.  Scratch needed: 64*nx*(4M2+1) bytes for pixel cells
 * (matrix-core passes; 64*nx*(4M2+1) with MVPB_PREC_SF_PLAIN64 too),
 * 64*ceil(n_edges/256)*(4M1+1)*(4M2+1) bytes for polygon cells; a request
 * above 16 MiB returns MVPB_E_NOMEM.  Every call on one GPU shares that
 * array, so calls that overlap in time on one GPU (two streams, two host
 * threads) race and must be serialised by the caller.  Returns after the
 * context stream has finished unless MVPB_F_ASYNC is passed. */
int mvpb_structure_factors_noalloc(mvpb_cell cell, int M1, int M2, int precision, double *F, unsigned flags);

/* Points equally spaced in arc length on Gamma(0,0)-X(1/2,0)-M(1/2,1/2)-Gamma
 * (the boundary of the irreducible zone of a square lattice), both ends
 * Gamma.  Q: host pointer, 2*n_k doubles. */
int mvpb_kpath_square(int n_k, double *Q);

/* n_k Bloch vectors equally spaced in arc length (measured in Cartesian k,
 * k = Q1 q^1 + Q2 q^2 with the reciprocal vectors of Sec. 2 for the lattice
 * rows h1, h2) along the polyline through the symmetry points named by
 * `path`, both ends included.  Letters (fractional coordinates):
 * G = (0, 0), X = (1/2, 0), Y = (0, 1/2), M = (1/2, 1/2) and J = (2/3, 1/3),
 * the zone corner of the hexagonal lattice h1 = a(1, 0), h2 = a(1/2, sqrt3/2).
 * "GXMG" is the square-lattice path of Sec. 5 (same points as
 * mvpb_kpath_square), "XGJX" the hexagonal path X-Gamma-J-X of Sec. 5.
 * n_k = 1 gives the first point.  Q: host pointer, 2*n_k doubles.  Unknown
 * letters, a path longer than 63 letters or a degenerate lattice:
 * MVPB_E_INVALID. */
int mvpb_kpath(const double lattice[4], const char *path, int n_k, double *Q);

/* Autotuning of the eigensolve's launch shape (per context and size class
 * of the operator order, n rounded up to a multiple of 128): the number of
 * independent stage-1 parts (streams), the number of consecutive
 * bulge-chasing sweeps dealt to one workgroup's wavefronts and the most
 * workgroups per item of the bulge chasing.  mvpb_autotune times the solve
 * of the plan's n_k points (Q as for mvpb_solve) under candidate shapes
 * (coordinate search from the defaults, median of three replays of the
 * captured launch sequence each, HIP events on the context stream; a
 * candidate replaces the best so far only if it is 2 % faster), keeps
 * the fastest for this context and, if cache_path is not NULL, merges it
 * into that JSON file (one entry per device name and size class).
 * *best_ms (nullable) receives its time.  The shapes change the schedule,
 * not the arithmetic: results are bitwise those of the defaults.
 * mvpb_ctx_load_tuning applies the file's entries for this context's device
 * (*n_loaded, nullable: how many); MVPB_E_INVALID for a missing file or a
 * malformed entry. */
int mvpb_autotune(mvpb_plan plan, int n_k, const double *Q, int n_bands, const char *cache_path,
                  double *best_ms);
int mvpb_ctx_load_tuning(mvpb_ctx ctx, const char *path, int *n_loaded);
/* The launch shape of the size class of operator order n, set explicitly
 * (parts 1..4, group 0 (= 8), 1, 2, 4 or 8, wg_max 0 (= 4) .. 4) or read
 * back (defaults 1, 0, 0 when the class has none). */
int mvpb_ctx_set_launch_shape(mvpb_ctx ctx, int n, int parts, int group, int wg_max);
int mvpb_ctx_get_launch_shape(mvpb_ctx ctx, int n, int *parts, int *group, int *wg_max);

/* Polls of a bounded hand-over wait of the bulge chasing before the point
 * gives up (its frequencies NaN, MVPB_E_DEVICE from host-pointer solves);
 * 0 restores the default (2^24).  The waits are bounded so that every
 * kernel exits even if a launch is not resident as planned; a small limit
 * forces the give-up path (used to test it). */
int mvpb_ctx_set_wait_limit(mvpb_ctx ctx, long long spins);

/* Plain device-to-device copy of `bytes` bytes (a multiple of 16, buffers
 * 16-byte aligned and not overlapping) by one kernel (copy16) on the context
 * stream; returns when it has finished.  It reads and writes each byte once,
 * which makes it the reference for calibrating hardware traffic counters
 * against a known byte count. */
int mvpb_copy_device(mvpb_ctx ctx, void *dst, const void *src, size_t bytes);

/* ---------------------------------------------------------------------------
 * Learned screening surrogate (not part of the paper's method).  A small
 * periodic CNN maps a binary 32 x 32 pixel cell (phase 1 = the stiff
 * inclusion material, phase 0 = the matrix) to 400 outputs: the lowest 10
 * bands at 40 k-points, normalised frequencies as supplied in the targets.
 * Layers: three-by-three circular convolutions 1->32 (stride 1), 32->32
 * (stride 2) x3, ReLU; fully connected 512->256 (ReLU) -> 400; mean squared
 * error; Adam (beta1 0.9, beta2 0.999, eps 1e-8).  Parameters are one flat
 * FP32 vector (conv weights [ky][kx][ci][co], dense weights [in][out], each
 * followed by its bias).  precision 0 runs every product in FP32, 1 on the
 * matrix cores with BF16 inputs and FP32 accumulation; master weights and
 * moments are FP32.  cells: batch*1024 bytes (0/1, row-major [32][32]),
 * target / out: batch*400 floats; host pointers unless MVPB_F_DEVICE_PTRS.
 * ------------------------------------------------------------------------- */
typedef struct mvpb_sur_s *mvpb_sur;
int mvpb_sur_create(mvpb_ctx ctx, int max_batch, int precision, uint64_t seed, mvpb_sur *out);
int mvpb_sur_destroy(mvpb_sur net);
int mvpb_sur_n_params(mvpb_sur net, int *n);
int mvpb_sur_get_params(mvpb_sur net, float *params);
int mvpb_sur_set_params(mvpb_sur net, const float *params);  /* also clears the Adam moments */
int mvpb_sur_infer(mvpb_sur net, int batch, const uint8_t *cells, float *out, unsigned flags);
/* loss and the gradient of the loss with respect to every parameter */
int mvpb_sur_gradients(mvpb_sur net, int batch, const uint8_t *cells, const float *target, float *loss,
                       float *grads, unsigned flags);
/* one Adam step on the batch; *loss (nullable) is the loss before the step */
int mvpb_sur_train_step(mvpb_sur net, int batch, const uint8_t *cells, const float *target, float lr,
                        float *loss, unsigned flags);
/* Checkpoint: the parameters, both Adam moments, the Adam step counter, the
 * product precision and the initialisation seed, written to the file `path`
 * (host-endian binary, a 40-byte header then 3 * n_params floats).
 * mvpb_sur_load creates a network on ctx for batches up to max_batch from
 * such a file; training continues exactly where the saved network stopped.
 * A file that is not such a checkpoint (or holds non-finite values):
 * MVPB_E_INVALID. */
int mvpb_sur_save(mvpb_sur net, const char *path);
int mvpb_sur_load(mvpb_ctx ctx, const char *path, int max_batch, mvpb_sur *out);

/* Kernel timers (diagnostics).  With profiling on, every kernel launch of a
 * context is bracketed by HIP events on the context stream and its device
 * time accumulated per kernel family.  Kernel ids: 0 structure_factors,
 * 1 toeplitz_scatter, 2 potrf_trtri, 3 zgemm, 4 combine_coefficients,
 * 5 form_operator, 6 he2hb_panel, 7 he2hb_hemm, 8 he2hb_wform,
 * 9 he2hb_her2k, 10 hb2st (the bulge chasing itself), 11 tridiag_eig,
 * 12 backtransform, 13 rayleigh_ritz, 14 hb2st_copy (band copy in and
 * tridiagonal out around hb2st) (MVPB_N_KERNELS in total).  Launches
 * inside the HIP graph of mvpb_solve_batch are not timed.
 * mvpb_ctx_profile(ctx, 1) clears the totals and starts timing, 0 stops.
 * mvpb_ctx_profile_read waits for the recorded events and returns the total
 * milliseconds, the number of launches and a static name string. */
#define MVPB_N_KERNELS 15
int mvpb_ctx_profile(mvpb_ctx ctx, int enable);
/* As mvpb_ctx_profile(ctx, 1), but only the kernels whose bit (1 << id) is
 * set in mask are bracketed by events (mask 0 stops timing), so that timing
 * one kernel family barely disturbs the rest. */
int mvpb_ctx_profile_mask(mvpb_ctx ctx, unsigned long long mask);
int mvpb_ctx_profile_read(mvpb_ctx ctx, int kernel, double *total_ms, long long *launches, const char **name);

#ifdef __cplusplus
}
#endif
#endif /* MVPB_H */
