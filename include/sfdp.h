/*
 * sfdp.h -- C ABI of the MI355X range-space Schur solver for
 * Poisson-constrained distributed optimal control.
 *
 * Method (Choi, Farhat, Murray, Saunders, arXiv 1312.5653):
 *   The discrete control problem of Sec. 2 (discrete QP) has the KKT system
 *       [ M   0     K ] [y  ]   [ M ybar   ]
 *       [ 0  beta M -M ] [u  ] = [ 0        ]
 *       [ K  -M     0 ] [lam]   [ -Kc yc   ]
 *   (the paper's phi is beta here and its volume matrix V is the consistent
 *   mass matrix M).  The range-space method (Sec. 3.1) solves
 *       S lam = Kc yc + K ybar,   S = K M^-1 K + M / beta,
 *   then y = ybar - M^-1 K lam and u = lam / beta.  S is applied through its
 *   exact complex factorization (Sec. 4)
 *       S = conj(Z) M^-1 Z,   Z = K + i alpha M,   alpha = beta^(-1/2),
 *   so one Schur solve is a solve with Z, a product with M, and a solve with
 *   conj(Z) done by conjugating the right-hand side and the result of a solve
 *   with Z.  Each Z solve is a FETI-DP domain decomposition solve (Sec. 5):
 *   subdomain factorizations, the corner coarse problem, and GMRES on the
 *   interface multipliers with the Dirichlet preconditioner.  On one GPU the
 *   subdomains are a batch.
 *
 * Problem class: the unit square (dim 2) or cube (dim 3), a uniform grid of
 * n_elem^dim Q1 cells, unit conductivity, Dirichlet data on the whole
 * boundary, split into (n_elem / sub_elem)^dim subdomains of sub_elem^dim
 * cells each.  Supported: dim 2 with 2 <= sub_elem <= 32; dim 3 with
 * 2 <= sub_elem <= 9 and at most 65535 subdomains; n_elem % sub_elem == 0
 * and n_elem / sub_elem >= 2.  In 3D the corners are the subdomain vertices
 * (no edge averages), a Delta node shared by k subdomains carries one
 * multiplier per pair (fully redundant), and 3D problems are solved through
 * the single-problem calls only (not sfdp_batch_* or the server).
 *
 * Dof numbering (all vectors):
 *   free node (i, j[, k]), 1 <= i, j, k <= n_elem - 1, has index
 *   (i-1) + (n_elem-1)(j-1) [+ (n_elem-1)^2 (k-1)]  (x fastest);
 *   boundary node has the index of its position among boundary nodes when
 *   all full-grid nodes (0..n_elem per axis) are visited with x fastest.
 *
 * Memory: every array argument is a DEVICE pointer on the context's GPU
 * (e.g. torch.Tensor.data_ptr() of a CUDA tensor), FP64, contiguous, owned by
 * the caller and accessed in stream order on the stream given at context
 * creation; the calls that take sfdp_opts accept host pointers instead when
 * opts->host_ptrs = 1 (staged by the library, the call then returns with the
 * outputs in host memory).  Complex vectors are interleaved (re, im) pairs.  Multiple
 * right-hand sides are stored one after another (column-major n x nrhs).
 * The library owns factors and workspaces; their device memory is charged
 * against the context's memory budget.
 *
 * Errors: every call returns an sfdp_status; nothing aborts or throws across
 * the ABI.  sfdp_last_error() returns a thread-local message for the last
 * failing call on the calling thread.  SFDP_E_INVALID: bad sizes, NULL
 * required pointers, beta <= 0 or not finite.  SFDP_E_STATE: solve before
 * sfdp_set_beta.  SFDP_E_NOMEM: the memory budget or the device ran out.
 * SFDP_E_NOCONV: the iteration limit was reached; outputs hold the last
 * iterate and info->rel_kkt its residual.  SFDP_E_DEVICE: a HIP error.
 *
 * Threading: a problem is used by one host thread at a time.
 */
#ifndef SFDP_H
#define SFDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfdp_ctx sfdp_ctx;
typedef struct sfdp_problem sfdp_problem;

typedef enum {
  SFDP_OK = 0,
  SFDP_E_INVALID = -1,
  SFDP_E_NOMEM = -2,
  SFDP_E_NOCONV = -3,
  SFDP_E_DEVICE = -4,
  SFDP_E_STATE = -5,
  SFDP_E_ADMIT = -6   /* a served request can never fit the context's memory budget */
} sfdp_status;

/* Arithmetic of the subdomain factors and of the interface operator.
 * SFDP_FP64:  complex128 everywhere.
 * SFDP_MIXED: subdomain line factors and interface operators (Z_rr^-1 on
 *             Delta, Phi) stored in complex64 and widened to FP64 as they
 *             are read; vectors, accumulation, the coarse problem, the
 *             Krylov orthogonalisation, the KKT residual and the outer
 *             iterative refinement in FP64.
 * SFDP_MIXED_IFACE: as SFDP_MIXED, but the subdomain line factors (the two
 *             full subdomain solves of every FETI-DP solve) in complex128.
 * In every mode the Dirichlet preconditioner's S_bb is stored in complex64. */
typedef enum { SFDP_FP64 = 0, SFDP_MIXED = 1, SFDP_MIXED_IFACE = 2 } sfdp_precision;

/* Solver controls; zero-initialised fields take the defaults in brackets. */
typedef struct {
  double tol_kkt;   /* stop when ||b - A x|| / ||b|| of the KKT system <= tol_kkt
                       [1e-10 FP64, 1e-8 MIXED] */
  double tol_inner; /* relative interface residual of each FETI-DP solve
                       [1e-8 FP64, 3e-7 MIXED; with complex64 operators GMRES
                       stagnates below about 5e-8]; see also tol_inner_first */
  int max_outer;    /* outer refinement steps [8] */
  int max_krylov;   /* GMRES iterations per FETI-DP solve, <= 400 [64]; the GMRES
                       kernel keeps per-iteration state for this many steps in
                       LDS, so a smaller cap leaves room to serve more
                       right-hand sides per launch (a solve that reaches the
                       cap is continued by the outer refinement) */
  int factors;      /* complex solves per refinement step [2]: 2 is the paper's
                       two-factor form (Z, then conj(Z) by conjugation); 1 uses
                       that the first factor alone determines the step:
                       Z (dy + i alpha dlam) = r3 + i alpha r1, so one FETI-DP
                       solve gives dy = Re, dlam = Im / alpha (the same result,
                       half the work; sfdp_apply_schur_inv then returns
                       -Im(Z^-1 r) / alpha) */
  int batch;        /* right-hand sides solved together, 1..4 [4]: each FETI-DP
                       launch sequence (subdomain solves, persistent GMRES)
                       serves up to this many right-hand sides in lockstep,
                       sharing every grid barrier and every pass over the
                       subdomain operators; results do not depend on it */
  int schur_block;  /* the S block of sfdp_apply_schur_inv and of the full-space
                       preconditioner [0]: 0 the exact S through its complex
                       factorization (Sec. 4); 1 the approximation
                       S_p = F M^-1 F, F = K + beta^-1/2 M, of Pearson and
                       Wathen (Sec. 3.2; S_p^-1 S has its eigenvalues in
                       [1/2, 1]).  S_p^-1 takes two FETI-DP solves with the
                       real factor F, whose factors a twin of the problem
                       holds (built on first use, and again after beta or the
                       coarse space changes; its memory counts against the
                       context's budget); opts->factors does not apply */
  double tol_inner_first; /* tol_inner of the first refinement step of
                       sfdp_solve_range_space and sfdp_batch_solve_range_space
                       [FP64: tol_inner; mixed: max(tol_inner, 1e-5)].  With
                       complex64 interface operators the first step ends near
                       a relative KKT residual of 5e-3 whether its solves stop
                       at 3e-7 or 1e-5, and the second step corrects it, so a
                       looser first solve saves GMRES iterations; set it to
                       tol_inner for the same tolerance in every step */
  int host_ptrs;    /* 1: the array arguments of the call are host pointers
                       (sfdp_solve_range_space, sfdp_solve_full_space,
                       sfdp_apply_schur_inv, sfdp_feti_solve,
                       sfdp_elastic_forward): the library copies the inputs
                       into a device buffer the problem keeps (grown on
                       demand, charged to the memory budget), runs the call
                       and copies the outputs back before returning [0:
                       device pointers].  SFDP_E_INVALID for other values */
} sfdp_opts;

/* Per-solve report. */
typedef struct {
  double rel_kkt;        /* final ||b - A x|| / ||b|| (FP64, on the GPU) */
  double rel_kkt_first;  /* the same after the first two-factor step */
  double imag_ratio;     /* ||Im lam_hat|| / ||Re lam_hat|| of the last factor-two solve */
  int outer_steps;       /* two-factor steps taken */
  int krylov_total;      /* GMRES iterations over all FETI-DP solves */
  int krylov_its[16];    /* per FETI-DP solve, in order (factor 1, factor 2, ...) */
  int n_feti;            /* FETI-DP solves done */
  int minres_its;        /* sfdp_solve_full_space: MINRES iterations over all
                            refinement steps (0 for the range-space calls) */
  double constr_viol;    /* relative constraint violation of the result (Sec. 6.2):
                            ||K y + Kc yc - M u|| / ||K y||, FP64 on the GPU */
  double eta_blk;        /* blockwise backward error of the result:
                            max_i ||r_i|| / (sum_j || |A_ij| |x_j| || + ||b_i||) over
                            the three block rows of the KKT system, |.| entrywise;
                            both metrics are -1 where not computed (served requests) */
  double t_setup_ms;     /* host time of the problem's last sfdp_set_beta (its
                            instance's set-up for batches; 0 for served requests) */
  double t_solve_ms;     /* host time of the call that produced this result (for
                            several targets per call: the whole call) */
} sfdp_info;

/* Launch-variant autotuning (enable = 1, the default): kernels with variants
 * that compute the same results in different launch shapes (the 2D subdomain
 * solve: one workgroup for all right-hand sides, one workgroup per right-hand
 * side, one wavefront per right-hand side, or one workgroup with a wavefront
 * per right-hand side and the line factors staged once; the 3D sweeps and
 * interface products: the depth of their load pipeline) time every variant on
 * the real operands the first time they run for a (kernel, shape, precision,
 * right-hand sides) key on a device, and keep the fastest for the process.
 * enable = 0 runs fixed defaults; enable = 2 + c (c = 0 .. 3) runs variant c
 * of every kernel that has it (the defaults elsewhere), for tests that compare
 * the variants.  Any call forgets the choices made so far.  Results do not
 * depend on the variant beyond the order of the floating-point sums (1e-12
 * relative).  SFDP_E_INVALID outside 0..5. */
sfdp_status sfdp_set_tuning(int enable);

/* Graph replay of refinement steps (enable = 1; default 0): a single 2D
 * problem's range-space refinement step (right-hand sides of both factors,
 * the FETI-DP solves with their persistent GMRES launches, the update and the
 * next KKT residual) is captured into a HIP graph the second time the same
 * step occurs (same active targets, caller arrays, inner tolerance and Krylov
 * limit) and replayed from then on; the host keeps the convergence test
 * between steps.  Captured steps are dropped when the problem's buffers, beta
 * or coarse space change.  Steps with kernel timing enabled run eagerly.
 * enable = 0 runs every step eagerly.  Results are bitwise the same either
 * way.  Off by default: a step's launches are queued ahead of the GPU anyway,
 * and the host's convergence test between steps stays, so replay does not
 * shorten a solve (measured at 512^2 on MI355X: 3.32 ms per call replayed from
 * the null stream, which replays through a capture stream of its own, against
 * 3.22 ms eagerly).
 * SFDP_E_INVALID for other values. */
sfdp_status sfdp_set_graphs(int enable);

/* Launch form of the persistent GMRES kernel in the range-space solves of a
 * single problem (sfdp_solve_range_space and its host-array form).  Its grid
 * barrier needs every workgroup resident at once.  mode = 1 (the default):
 * a plain launch whose workgroups first count themselves on a device word and
 * wait, bounded, until all have arrived; if they do not (other work holds the
 * compute units), every workgroup returns without work, the refinement step
 * leaves the iterate unchanged (the update kernel sees the flag) and runs
 * again with cooperative launches, which that problem then keeps.  mode = 0:
 * cooperative launches always (hipLaunchCooperativeKernel guarantees
 * co-residency, at ~11 us of idle device before and after each launch on
 * MI355X).  mode = 2: as 1 with no wait in the check, so that the fallback
 * runs (for tests).  Results are the same in every mode.  Batches and the
 * other entry points always launch cooperatively.  SFDP_E_INVALID for other
 * values. */
sfdp_status sfdp_set_gmres_launch(int mode);

/* Arithmetic of the subdomain line factorization and line solves of the
 * set-up (Sec. 4 factors, the local solves of Sec. 5) for problems with
 * complex64 storage (SFDP_MIXED), from the next sfdp_set_beta (or batch
 * set-up) on: bits = 64 (the default) computes them in FP64 on the FP64 matrix
 * cores and rounds the stored factors to complex64 once; bits = 32 computes
 * them in complex64 on the FP32 matrix cores (v_mfma_f32_16x16x4f32, FP32
 * accumulation).  The interface Schur complements' inverses, the coarse
 * problem and every solve stay FP64.  Other precisions always use 64.
 * SFDP_E_INVALID for other values. */
sfdp_status sfdp_set_setup_arithmetic(int bits);

/* Sizes of a problem. */
typedef struct {
  int64_t n_free;        /* unconstrained dofs (n_elem-1)^dim */
  int64_t n_bdry;        /* Dirichlet dofs */
  int64_t n_sub;         /* subdomains */
  int64_t n_mult;        /* interface multipliers */
  int64_t n_corner;      /* corner dofs */
  int64_t max_delta;     /* largest number of interface (Delta) dofs of a subdomain */
  int64_t resident_bytes;/* device bytes held by the problem after sfdp_set_beta */
  int64_t n_coarse;      /* coarse unknowns in use: corners, plus one per interface edge
                            when the coarse space is edge-augmented (the default) */
} sfdp_sizes;

/* Create a context on HIP device `device`; all work is ordered on `stream`
 * (a hipStream_t, NULL for the default stream).  mem_budget_bytes = 0 means
 * no limit beyond the device's memory. */
sfdp_status sfdp_ctx_create(int device, size_t mem_budget_bytes, void* stream, sfdp_ctx** out);
/* Frees the context.  Problems, batches and servers keep a pointer to their
 * context, so it refuses with SFDP_E_STATE (and frees nothing) while any of
 * them is alive: destroy those first.  NULL is a no-op (SFDP_OK). */
sfdp_status sfdp_ctx_destroy(sfdp_ctx* ctx);
const char* sfdp_last_error(void);
/* Revision of the structures and calls declared here: 2 since
 * sfdp_opts.host_ptrs (host arrays staged by the library).  A binding reads it
 * before relying on something a library built from older sources lacks (an
 * older library would take host addresses for device ones). */
int sfdp_abi_version(void);

/* Set up the mesh, the subdomain partition and the interface maps (Sec. 5:
 * signed Boolean matrices, corners) for the problem class described above. */
sfdp_status sfdp_problem_create(sfdp_ctx* ctx, int dim, int n_elem, int sub_elem,
                                sfdp_precision prec, sfdp_problem** out);
sfdp_status sfdp_problem_sizes(const sfdp_problem* p, sfdp_sizes* out);
void sfdp_problem_destroy(sfdp_problem* p);

/* Coarse space of the FETI-DP solves (Sec. 5; the augmentation compared in
 * Table 1).  edge_averages = 1: the corners plus one average per interface
 * edge, the constraint Q^T B_r u_r = 0 (Q: one column of ones on the
 * multipliers of each edge) enforced exactly at every Krylov iterate through
 * the extra coarse unknowns; 0: corners only.  The solution is the same; the
 * iteration counts differ.  Default: edge averages while the augmented coarse
 * problem has at most 1024 unknowns (up to 19 x 19 subdomains), corners only
 * beyond (its dense inverse would dominate the set-up).  Takes effect at the
 * next sfdp_set_beta (the problem must be set up again: SFDP_E_STATE until then).
 * SFDP_E_INVALID for values other than 0 and 1. */
sfdp_status sfdp_set_coarse_space(sfdp_problem* p, int edge_averages);

/* Fix beta (Sec. 2 regularisation) and build the FETI-DP operators of
 * Z = K + i beta^(-1/2) M (Sec. 4 factor, Sec. 5 solver): per subdomain the
 * factorization of the remainder block, its interface Schur complement and
 * its inverse, the corner condensation; then the coarse matrix and its
 * inverse.  The factors stay resident until the next call or destroy. */
sfdp_status sfdp_set_beta(sfdp_problem* p, double beta);

/* Range-space solve (Sec. 3.1 with the Sec. 4 factorization) for nrhs targets.
 *   ybar: n_free x nrhs    target state at the free nodes
 *   yc:   n_bdry x nrhs    Dirichlet data, or NULL for zero
 *   y, u, lam: n_free x nrhs outputs (state, control, adjoint).
 * Starts from (y, u, lam) = (ybar, 0, 0), whose KKT residual is
 * (0, 0, -(K ybar + Kc yc)); every step applies the two complex factors to
 * the current FP64 KKT residual (r1, r2, r3):
 *   dw = Z^-1 (-r3 - i alpha r1);  v = r1 + M dw;
 *   dlam = Re conj(Z^-1 conj(v));  dy = -Re dw;  u = lam / beta.
 * The first step is the paper's range-space solve with the real right-hand
 * side b = K ybar + Kc yc; later steps are iterative refinement.
 * Targets are taken in groups of opts->batch; the unfinished members of a
 * group take each step together and each stops on its own test.
 * opts and info may be NULL; info, if given, has nrhs entries.
 * Returns SFDP_E_NOCONV (after finishing all targets) if any target missed
 * tol_kkt within max_outer steps. */
sfdp_status sfdp_solve_range_space(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                                   double* y, double* u, double* lam, const sfdp_opts* opts,
                                   sfdp_info* info);

/* z = S^-1 r for real r (n_free x nrhs), through the two complex factors
 * (Sec. 4): z = Re conj(Z^-1 conj(M Z^-1 r)).  This is the S block of the
 * block-diagonal preconditioner of Sec. 3.2.  With opts->schur_block = 1,
 * z = S_p^-1 r = F^-1 M F^-1 r instead (Sec. 3.2, F = K + beta^-1/2 M).
 * info, if given, has nrhs entries (two FETI-DP solves each). */
sfdp_status sfdp_apply_schur_inv(sfdp_problem* p, int nrhs, const double* r, double* z,
                                 const sfdp_opts* opts, sfdp_info* info);

/* One FETI-DP solve (Sec. 5) of Z x = f (conj_z = 0) or conj(Z) x = f
 * (conj_z = 1); f and x are complex n_free x nrhs, interleaved. */
sfdp_status sfdp_feti_solve(sfdp_problem* p, int conj_z, int nrhs, const double* f, double* x,
                            const sfdp_opts* opts, int* krylov_its);

/* Full-space method (Sec. 3.2): the KKT system A x = b solved by MINRES with
 * the block-diagonal preconditioner P_mgw = blkdiag(V, phi V, S) (Murphy,
 * Golub and Wathen: P_mgw^-1 A has at most three distinct eigenvalues), with
 * V^-1 exact (Kronecker product of 1D tridiagonal solves) and S^-1 through
 * the complex factorization (as sfdp_apply_schur_inv: opts->tol_inner and
 * opts->factors apply; opts->schur_block = 1 puts the approximation S_p of
 * Pearson and Wathen in place of S, the comparison of Table 7), inside FP64
 * iterative refinement on the KKT residual: each refinement step runs MINRES
 * on A dx = b - A x to a relative preconditioned residual of 1e-6 (at most 30
 * iterations with S, 100 with S_p).  Arguments,
 * layout, the start (ybar, 0, 0) and the stopping test (opts->tol_kkt) are
 * those of sfdp_solve_range_space; right-hand sides are solved one after
 * another.  info->outer_steps counts refinement steps, info->minres_its the
 * MINRES iterations, info->n_feti and info->krylov_* the FETI-DP solves.
 * Requires n_elem <= 1025. */
sfdp_status sfdp_solve_full_space(sfdp_problem* p, int nrhs, const double* ybar, const double* yc, double* y,
                                  double* u, double* lam, const sfdp_opts* opts, sfdp_info* info);

/* FP64 products with the assembled matrices (Sec. 2): which = 'K' gives
 * y = K x + Kc xc (xc may be NULL), 'M' gives y = M x, 'I' gives y = M^-1 x
 * (the V block of the full-space preconditioner; n_elem <= 1025).  x, y:
 * n_free x nrhs real; xc: n_bdry x nrhs. */
sfdp_status sfdp_apply_operator(sfdp_problem* p, char which, int nrhs, const double* x,
                                const double* xc, double* y);

/* Relative KKT residual ||b - A x|| / ||b|| of (y, u, lam) in FP64 (Sec. 2
 * KKT system), one value per right-hand side written to rel (host array). */
sfdp_status sfdp_kkt_residual(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                              const double* y, const double* u, const double* lam, double* rel);

/* The same relative KKT residuals as sfdp_kkt_residual, computed without any
 * allocation: for callers that cannot allocate device or pinned memory (code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * It calls no hipMalloc, hipFree or allocating library routine; its partial
 * sums live in a fixed device array of 512 KiB (65,536 doubles) per device,
 * held until the process ends.  Limit: one call handles up to 4 right-hand
 * sides at a time and needs 16 + 8 ceil(n_free / 256) doubles, so n_free must be
 * at most 2,096,640 (2D meshes up to 1448 x 1448 cells, 3D up to 128^3);
 * beyond it the call returns SFDP_E_INVALID.  ybar, yc, y, u, lam as for
 * sfdp_kkt_residual (device arrays); rel is a DEVICE array of nrhs doubles,
 * written in stream order on the context's stream (the call does not wait).
 * Every call on one device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (other threads, other streams) race
 * and must be serialised by the caller.  Errors: SFDP_E_INVALID (NULL
 * argument, nrhs <= 0, mesh over the limit), SFDP_E_STATE (beta not set),
 * SFDP_E_DEVICE (launch failure). */
sfdp_status sfdp_kkt_residual_noalloc(sfdp_problem* p, int nrhs, const double* ybar, const double* yc,
                                      const double* y, const double* u, const double* lam, double* rel);

/* Inspection of the resident FETI-DP operators, for testing.  Writes FP64
 * complex (interleaved) values to the device array out, row-major:
 *   SFDP_Q_SINV  sub s: n_d x n_d  (Z_rr^-1 restricted to the subdomain's
 *                Delta dofs, in increasing local node index a + (m+1) b
 *                [+ (m+1)^2 c]; n_d is returned in *rows and *cols);
 *   SFDP_Q_SBB   sub s: n_d x n_d  interface Schur complement (Sec. 5, S_bb);
 *   SFDP_Q_PHI   sub s: n_d x n_c  coarse basis on Delta rows: Z_rr^-1 Z_rc
 *                for the subdomain's corners (increasing local index), then,
 *                when edge-augmented, Z_rr^-1 B_r^T q_e for its edges in the
 *                order left, right, bottom, top side;
 *   SFDP_Q_COARSE     : n_coarse x n_coarse coarse matrix: K_cc*, or with edge
 *                averages [[K_cc*, -F_rc^T Q], [-Q^T F_rc, -Q^T F_rr Q]] over
 *                the corners (increasing node id) then the edges (increasing
 *                pair of adjacent subdomains);
 *   SFDP_Q_COARSE_INV : its inverse as used by the solves (Gauss-Jordan
 *                without pivoting, corners first);
 * (3D: the same queries; the corners of SFDP_Q_PHI are the non-Dirichlet
 * vertices of the subdomain in increasing local index.)
 * out may be NULL to query the shape only. */
typedef enum { SFDP_Q_SINV = 0, SFDP_Q_SBB = 1, SFDP_Q_PHI = 2, SFDP_Q_COARSE = 3, SFDP_Q_COARSE_INV = 4 } sfdp_query;
sfdp_status sfdp_inspect(sfdp_problem* p, sfdp_query what, int sub, double* out, int* rows, int* cols);

/* Interface-level products for testing, on multiplier vectors (complex,
 * interleaved, length n_mult; multipliers ordered by the full id of their
 * node, then by the pair of subdomains (s_a < s_b), signed +1 on s_a):
 *   which = 'F': y = F_DP x (Sec. 5 interface operator with the coarse
 *                correction);  which = 'P': y = P^-1 x (Dirichlet
 *                preconditioner);  which = 'D': y = d(f) for the complex
 *                free-node load x (length n_free) -- the FETI-DP
 *                right-hand side. */
sfdp_status sfdp_interface_apply(sfdp_problem* p, char which, const double* x, double* y);

/* ---- Linear elasticity: the solid cantilever control of Sec. 6.2 ----
 *
 * The state equation is the elastostatic one: K is the stiffness of an
 * isotropic linear-elastic solid (Young's modulus E, Poisson's ratio nu) on
 * trilinear elements with three displacement dofs per node, M (the paper's V)
 * the consistent vector mass, the control a body force.  The body is the box
 * [0, length] x [0, 1] x [0, 1] of n cells per unit length, clamped on the
 * face x = 0 (homogeneous, so there is no Kc and no yc: pass NULL), free
 * elsewhere, cut into (length n / sub_elem) x (n / sub_elem)^2 cubic
 * subdomains of sub_elem^3 cells (2 <= sub_elem <= 6, at most 65535
 * subdomains).  FETI-DP (Sec. 5) takes the three dofs of every unclamped
 * subdomain vertex as corner unknowns, one multiplier per pair of subdomains
 * sharing an interface node per component (fully redundant), the
 * multiplicity-scaled Dirichlet preconditioner, and dense subdomain inverses
 * (blocked Gauss-Jordan on the device).
 *
 * Dofs: grid node (i, j, k), 0 <= i <= length n, 0 <= j, k <= n; the free
 * nodes (i >= 1) are numbered x fastest, f = (i-1) + length n (j + (n+1) k),
 * and free dof 3 f + c holds displacement component c (0: x, 1: y, 2: z).
 * n_free = 3 length n (n+1)^2.  Multipliers are ordered by free dof, then by
 * the pair of subdomains (s_a < s_b), +1 on s_a; corners (coarse unknowns) are
 * the unclamped vertex nodes in increasing grid index, three dofs each.
 *
  * E = 0 or nu = 0 take the paper's rubber (E = 20.7 MPa, nu = 0.45).  The
 * handle is an sfdp_problem: sfdp_set_beta, sfdp_solve_range_space,
 * sfdp_apply_schur_inv, sfdp_feti_solve, sfdp_apply_operator ('K', 'M'),
 * sfdp_kkt_residual, sfdp_inspect (SFDP_Q_SINV / SBB rows and columns in
 * increasing local dof 3 l + c, l = a + (m+1) b + (m+1)^2 c; SFDP_Q_PHI columns
 * the unclamped vertex dofs in increasing local dof), sfdp_interface_apply,
 * sfdp_problem_sizes and sfdp_problem_destroy apply; the batch, the server,
 * the full-space method, edge averages, the one-factor form and
 * sfdp_kkt_residual_noalloc do not (SFDP_E_INVALID).
 *
 * Stopping test of sfdp_solve_range_space on these problems: the blockwise
 * backward error eta_blk <= opts->tol_kkt [1e-12 FP64, 1e-10 mixed], not the
 * relative KKT residual: the right-hand side (M ybar, 0, 0) is many orders of
 * magnitude below the stiffness terms of the residual (E / h^2 against h^3),
 * so even the exact solution's ||b - A x|| / ||b|| is about 1e-7 in FP64.
 * info->rel_kkt still reports that residual.  max_krylov defaults to 300; the
 * first step's inner tolerance defaults to tol_inner. */
sfdp_status sfdp_elastic_create(sfdp_ctx* ctx, int n, int sub_elem, int length, double young, double poisson,
                                sfdp_precision prec, sfdp_problem** out);

/* f (device, n_free) = the consistent nodal forces of a uniform pressure on
 * the bottom face z = 0 pushing in -z (Sec. 6.2 uses 100 kPa = 1e5): each
 * bottom face cell gives each of its unclamped vertices -pressure h^2 / 4. */
sfdp_status sfdp_elastic_pressure_load(sfdp_problem* p, double pressure, double* f);

/* Forward elastostatic solve u = K^-1 f (Sec. 6.2: the target state is the
 * displacement under the pressure load) for nrhs real right-hand sides
 * (device, n_free x nrhs), by FETI-DP on K alone with complex128 factors
 * whatever the problem's precision: they are built on the first call (a
 * twin of the partition holds them, charged to the context's budget) and kept
 * until the problem is destroyed; beta need not be set.  opts->tol_inner is
 * the relative interface residual [1e-8], krylov_its (optional, host) gets
 * the GMRES iterations per right-hand side. */
sfdp_status sfdp_elastic_forward(sfdp_problem* p, int nrhs, const double* f, double* u, const sfdp_opts* opts,
                                 int* krylov_its);

/* ---- Batches of independent instances (uneven sizes, one beta each) ----
 *
 * A batch holds `count` 2D instances of the problem class above, instance i
 * with n_elem[i] cells per side, all with the same sub_elem and precision.
 * Every step of the set-up and of the solve runs over all instances in one
 * launch per kernel: the subdomains of all instances form one batch, and the
 * interface GMRES of every instance runs inside a shared persistent
 * cooperative launch, each instance with its own Krylov state, reductions and
 * grid barrier over its share of the blocks (instances whose blocks do not all
 * fit on the device at once are split over consecutive such launches).
 * Results are those of solving each instance on its own with the same options. */
typedef struct sfdp_batch sfdp_batch;
sfdp_status sfdp_batch_create(sfdp_ctx* ctx, int count, const int* n_elem, int sub_elem,
                              sfdp_precision prec, sfdp_batch** out);
void sfdp_batch_destroy(sfdp_batch* b);
/* Sizes of instance i (as sfdp_problem_sizes). */
sfdp_status sfdp_batch_sizes(const sfdp_batch* b, int i, sfdp_sizes* out);
/* Factor every instance for its beta[i] (host array of count values), as
 * sfdp_set_beta does for one problem. */
sfdp_status sfdp_batch_set_beta(sfdp_batch* b, const double* beta);
/* The set-up operators of instance i after sfdp_batch_set_beta, as sfdp_inspect
 * returns them for one problem (same queries, shapes and errors); a batch may
 * take other set-up paths than a lone problem (the coarse inverse of several
 * mid-size instances, one workgroup each). */
sfdp_status sfdp_batch_inspect(sfdp_batch* b, int i, sfdp_query what, int sub, double* out, int* rows,
                               int* cols);
/* Range-space solves (as sfdp_solve_range_space) of nrhs[i] targets of
 * instance i.  ybar, yc, y, u, lam are host arrays of count device pointers
 * (each as in sfdp_solve_range_space; yc or yc[i] may be NULL for zero
 * Dirichlet data; pointers of instances with nrhs[i] = 0 are not read).
 * info, if given, has sum(nrhs) entries, instance by instance. */
sfdp_status sfdp_batch_solve_range_space(sfdp_batch* b, const int* nrhs, const double* const* ybar,
                                         const double* const* yc, double* const* y, double* const* u,
                                         double* const* lam, const sfdp_opts* opts, sfdp_info* info);

/* ---- Serving: continuous batching of requests ----
 *
 * A server owns a worker thread that uses the context's stream (the caller
 * must not use that context from other threads meanwhile).  Requests (one
 * mesh, one beta, nrhs targets) are admitted while the context's memory
 * budget allows: a request joins the resident instance of its (mesh, beta)
 * or a new instance is created and factored (new instances admitted together
 * are factored in shared set-up passes whose scratch stays under 1/16 of the
 * budget, 4 GiB without one, unless a single instance needs more; the
 * scratch pool stays with the context); idle instances are evicted, least
 * recently used first, when memory is short, and a request that does not fit
 * waits until memory frees.  Every instance serves up to four targets at a
 * time in slots; each worker tick gives every occupied slot of every resident
 * instance one KKT residual and, if not converged, one two-factor refinement
 * step, all instances in one launch per kernel (the batch path above).
 * Targets that finish free their slots, and waiting targets take free slots
 * at the next tick, so requests that arrive while others run join them on
 * the device.  A result does not depend on what else is in flight (up to the
 * rounding of multiply-add contraction, 1e-12 relative).
 * 3D requests and full-space requests (mode 1) take a solo lane: after each
 * tick the worker solves one of them whole, in arrival order, on a resident
 * single problem of its (dim, mesh, beta) (at most two are kept, least
 * recently used dropped first; on a memory shortage the idle batched
 * instances are evicted and the set-up tried once more, else the request is
 * refused with SFDP_E_ADMIT). */
typedef struct sfdp_server sfdp_server;
typedef struct {
  int dim;           /* 2 or 3 */
  int n_elem;        /* cells per side */
  int sub_elem;      /* cells per subdomain side */
  double beta;
  int nrhs;          /* targets */
  const double* ybar;  /* device, n_free x nrhs (as sfdp_solve_range_space) */
  const double* yc;    /* device, n_bdry x nrhs, or NULL for zero */
  double *y, *u, *lam; /* device outputs, n_free x nrhs; all arrays stay valid until polled */
  int mode;          /* 0: range-space method; 1: full-space method (sfdp_solve_full_space) */
} sfdp_request;
typedef struct {
  int64_t submitted, completed, failed;
  int64_t setups;      /* instances factored */
  int64_t evictions;   /* instances evicted for memory */
  int64_t ticks;       /* worker steps */
  int64_t resident;    /* instances resident now */
  int64_t device_bytes;/* device memory held by the context */
  double mean_ms, p50_ms, p99_ms;  /* latency (submit to result) of completed requests */
  int64_t solo_in_flight_max;  /* most 3D / full-space requests advancing together so far */
} sfdp_server_info;
/* opts as for sfdp_solve_range_space (batch is not used: slots hold up to 4). */
sfdp_status sfdp_server_create(sfdp_ctx* ctx, sfdp_precision prec, const sfdp_opts* opts,
                               sfdp_server** out);
/* Queue a request (returns at once) and its ticket. */
sfdp_status sfdp_server_submit(sfdp_server* s, const sfdp_request* req, uint64_t* ticket);
/* SFDP_E_STATE while pending when wait = 0; otherwise waits.  On completion
 * returns the request's status (SFDP_OK, SFDP_E_NOCONV, SFDP_E_ADMIT when it
 * can never fit the budget, SFDP_E_DEVICE), fills info[nrhs] and the latency
 * (milliseconds from submit to result) if given, and releases the ticket. */
sfdp_status sfdp_server_poll(sfdp_server* s, uint64_t ticket, int wait, sfdp_info* info,
                             double* latency_ms);
sfdp_status sfdp_server_stats(sfdp_server* s, sfdp_server_info* out);
/* Finishes every admitted and pending request, then stops. */
void sfdp_server_destroy(sfdp_server* s);

/* Kernel timing with HIP events recorded on the context's stream around the
 * launches of the two hot kernels of every FETI-DP solve: the persistent
 * interface GMRES kernel and the batched subdomain solve kernel (two launches
 * per FETI-DP solve).  enable = 1 records both, enable = 2 the GMRES launches
 * only, enable = 0 stops; 1 and 2 clear the totals.  sfdp_kernel_times reports
 * totals in milliseconds, launch counts and the GMRES iterations done by the
 * timed launches.  Timing adds one event pair per timed launch (on MI355X each
 * event record leaves the device idle ~6 us) and is meant for measurement
 * runs.  SFDP_E_INVALID outside 0..2. */
typedef struct {
  double gmres_ms;        /* summed duration of the GMRES kernel launches */
  double local_ms;        /* summed duration of the subdomain solve launches */
  int64_t gmres_launches;
  int64_t gmres_iters;    /* loop trips summed over the timed GMRES launches (a launch
                             serving several right-hand sides runs as many trips as
                             its slowest one needs) */
  int64_t local_launches;
  int64_t gmres_rhs_iters;/* iterations summed over right-hand sides */
  int gmres_width;        /* right-hand sides per GMRES launch of the last solve
                             (the widest kernel of 4, 2, 1 whose LDS fits) */
  int gmres_resident;     /* 1 if that launch kept the Schur blocks in LDS */
} sfdp_timing;
sfdp_status sfdp_timing_enable(sfdp_problem* p, int enable);
sfdp_status sfdp_kernel_times(sfdp_problem* p, sfdp_timing* out);

#ifdef __cplusplus
}
#endif
#endif /* SFDP_H */
