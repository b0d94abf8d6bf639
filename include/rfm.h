/*
 * rfm.h -- C ABI of the MI355X (gfx950) hot path of block sigma-RRQR filtering and
 * right-preconditioned LSQR for ELM-FBPINN least-squares systems.
 *
 * The method (van Beek, Dolean, Moseley, "Local feature filtering for scalable and
 * well-conditioned domain-decomposed random feature methods"):
 *   - the weighted least-squares system min ||M a - h|| of eq. ELMFBPINN_ls, with
 *     M = sum_j V_j^T M_j W_j block-sparse over overlapping subdomains (eq. DomainDecomp);
 *   - every block M_j is filtered by a sigma-RRQR factorisation (Algorithm 1), the
 *     threshold taken relative to the leading diagonal entry of R_j;
 *   - the filtered system is right-preconditioned by S^{-1} = sum_j W_j^T R_j^{-1} W_j,
 *     which makes M_hat S^{-1} = sum_j V_j^T Q_hat_j W_hat_j (Proposition 3.1), and solved
 *     by LSQR; a = S^{-1} y with zeros at the dropped columns (Algorithm 2).
 *
 * Conventions shared by every call:
 *   - "device" pointers are HIP device memory (gfx950) owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library keeps no
 *     allocation between calls, except where a call says otherwise.
 *   - Every call validates its arguments on the host before launching anything; on
 *     RFM_EINVAL / RFM_EUNSUPPORTED no output has been touched.  On RFM_EHIP outputs
 *     are undefined.  rfm_last_error() returns a description of the last failure on
 *     the calling thread.
 *   - Calls taking a stream enqueue their work on it and return without waiting,
 *     unless marked (sync).
 *   - Floating point is IEEE binary64 throughout this header.
 */
#ifndef RFM_H
#define RFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RFM_OK = 0,
  RFM_EINVAL = 1,         /* invalid argument (null pointer, bad size, inconsistent layout) */
  RFM_EHIP = 3,           /* a HIP runtime call failed */
  RFM_ENOTCONV = 4,       /* LSQR reached maxit; outputs hold the last iterate */
  RFM_EUNSUPPORTED = 5    /* sizes beyond what the kernels are built for */
} rfm_status;

/* Element types of operand copies (the precision form). */
typedef enum {
  RFM_F64 = 0,            /* IEEE binary64                                           */
  RFM_F32 = 1,            /* IEEE binary32, rounded to nearest even from binary64      */
  RFM_BF16 = 2            /* bfloat16 (upper 16 bits of binary32), the binary32 value
                             rounded to nearest even                                 */
} rfm_dtype;

/* Row operators (the linear PDE / boundary operators N and B_l of Section 2.1).
 * Inputs x have d coordinates; for RFM_OP_HEAT the last coordinate is time.
 * RFM_OP_COEF + i applies operator i of the problem's coefficient table (opcoef):
 *   c0 u + sum_i (c1_i d_i u + c2_i d_ii u),
 * which covers the paper's own problems (Section 5.1): the damped oscillator
 * m u'' + mu u' + k u and its initial velocity u'(0), and the wave operator
 * sum_{i<d-1} d_ii u - c^-2 d_tt u.  A code that is none of these, or a table index out of
 * range, is read as RFM_OP_VALUE. */
typedef enum {
  RFM_OP_NEG_LAPLACE = 0, /* -sum_i d_ii u                          */
  RFM_OP_HEAT = 1,        /* d_t u - kappa * sum_{i<d-1} d_ii u       */
  RFM_OP_HELMHOLTZ = 2,   /* sum_i d_ii u + ksq * u                   */
  RFM_OP_VALUE = 3,       /* u (Dirichlet and initial-condition rows)  */
  RFM_OP_COEF = 16        /* + i: constant-coefficient operator i of opcoef */
} rfm_rowop;

/* Block layout of the global matrix (eq. DomainDecomp).  Produced on the host by
 * rfm_plan; the caller copies the arrays to the device and fills the pointers.
 *   I_j  = rows r with |x_r,i - mu_j,i| < hw_j,i for every i (open support of the
 *          window), ascending;
 *   block j of M, Q: column-major |I_j| x K_j at element offset blk_off[j]
 *          (column k = local feature k, leading dimension |I_j|);
 *   block j of R:    column-major K_j x K_j at element offset rsq_off[j];
 *   per-feature vectors (kept, y, a): entry (j,k) at feat_off[j] + k. */
typedef struct {
  int32_t d;              /* input dimension (1..3)                          */
  int32_t J;              /* number of subdomains                           */
  int64_t N;              /* rows of the global system                      */
  int64_t nnz_rows;       /* sum_j |I_j|                                    */
  int64_t nnz;            /* sum_j |I_j| K_j                                */
  int64_t ncols;          /* sum_j K_j                                      */
  int64_t nrsq;           /* sum_j K_j^2                                    */
  int32_t max_rows;       /* max_j |I_j|                                    */
  int32_t max_cols;       /* max_j K_j                                      */
  const int64_t *row_off; /* device [J+1] prefix sums of |I_j|              */
  const int32_t *rows;    /* device [nnz_rows] global row ids, block-major  */
  const int32_t *inc_blk; /* device [nnz_rows] block id of each incidence   */
  const int64_t *rinc_off;/* device [N+1] per-row incidence ranges          */
  const int64_t *rinc;    /* device [nnz_rows] incidence ids per row, ascending j */
  const int64_t *feat_off;/* device [J+1] prefix sums of K_j                */
  const int64_t *blk_off; /* device [J+1] prefix sums of |I_j| K_j          */
  const int64_t *rsq_off; /* device [J+1] prefix sums of K_j^2              */
} rfm_layout;

/* Activation Xi of the random features (eq. fcn_depth_h).  tanh is the baseline of every
 * problem in Section 5; the ablation rows of its three results tables use the sigmoid and
 * sin instead. */
typedef enum {
  RFM_ACT_TANH = 0,       /* tanh(s)                                        */
  RFM_ACT_SIGMOID = 1,    /* 1 / (1 + exp(-s))                              */
  RFM_ACT_SIN = 2         /* sin(s)                                         */
} rfm_activation;

/* Discretised problem (Section 2.1 and Section 4.2): subdomain geometry, random
 * features phi_jk = act(w_jk . (x - mu_j)/hw_j + b_jk) (eq. fcn_depth_h, depth 1,
 * inputs normalised to [-1,1] per subdomain), points and per-row data.
 * With depth h > 1 each subdomain's features share h-1 hidden layers
 *   z0 = (x - mu_j)/hw_j,  z_l = act(W_l z_{l-1} + b_l),  phi_jk = act(w_jk . z_{h-1} + b_jk).
 * A hard-constraint ansatz (Section 5.1: u~ = g u_hat, after Lagaris et al.) is given by its
 * factor g per point: ansatz [N*(1+2d)] holds, for point r, g, d_i g (i < d) and d_ii g
 * (i < d) at offset r*(1+2d); the row operators then apply to g u_hat (product rule), and
 * rfm_evaluate returns g u_hat.  An additive part of an ansatz belongs in rhs. */
typedef struct {
  const double *x;        /* device [N*d] row-major points                 */
  const int32_t *rowop;   /* device [N] rfm_rowop per row                  */
  const double *weight;   /* device [N] row scale s_r (1/sqrt(N_I), sqrt(lambda_l/N_B^(l))) */
  const double *rhs;      /* device [N] unscaled right-hand side f or g_l  */
  const double *mu;       /* device [J*d] subdomain centres                */
  const double *hw;       /* device [J*d] subdomain half-widths            */
  const double *w;        /* device [ncols*d] feature weights              */
  const double *b;        /* device [ncols] feature biases                 */
  double kappa;           /* RFM_OP_HEAT diffusion constant                */
  double ksq;             /* RFM_OP_HELMHOLTZ k^2                          */
  int32_t activation;     /* rfm_activation of the features (0 = tanh)     */
  int32_t nopcoef;        /* rows of opcoef (0: no table)                  */
  const double *opcoef;   /* device [nopcoef*(1+2d)]: per operator c0, c1_0..c1_{d-1},
                             c2_0..c2_{d-1}; nullable when nopcoef = 0      */
  const double *ansatz;   /* device [N*(1+2d)] g, d_i g, d_ii g per point, or NULL (g = 1) */
  int32_t depth;          /* h of eq. fcn_depth_h: 0 or 1 = features on the input, 2..8 =
                             h-1 hidden layers of width `hidden` shared by a subdomain's
                             features, which then act on the last hidden layer            */
  int32_t hidden;         /* width H of the hidden layers (1..16) when depth > 1           */
  const double *net;      /* device, when depth > 1: per subdomain j, at offset
                             j*(H*d + H + (depth-2)*(H*H + H)), layer 1 W [H x d] row-major
                             then b [H], then layers 2..depth-1 W [H x H] row-major then b [H];
                             w is then [ncols*H] (feature weights on the last hidden layer) */
} rfm_problem;

/* Planning (sync, host only).  Builds the supports I_j of eq. DomainDecomp from host
 * copies of the points (x [N*d]), centres and half-widths (mu, hw [J*d]) and the
 * feature counts (K [J]).  Membership uses the strict test |x - mu| < hw in binary64.
 * Call once with all array outputs NULL to get the sizes in *sizes_out
 * ([0]=nnz_rows, [1]=nnz, [2]=ncols, [3]=nrsq, [4]=max_rows, [5]=max_cols); then call
 * again with arrays of those sizes: row_off, feat_off, blk_off, rsq_off [J+1],
 * rows, inc_blk, rinc [nnz_rows], rinc_off [N+1]. */
rfm_status rfm_plan(int32_t d, int32_t J, int64_t N, const double *x, const double *mu,
                    const double *hw, const int32_t *K, int64_t *sizes_out,
                    int64_t *row_off, int32_t *rows, int32_t *inc_blk, int64_t *rinc_off,
                    int64_t *rinc, int64_t *feat_off, int64_t *blk_off, int64_t *rsq_off);

/* Bytes of device workspace rfm_assemble needs for this layout. */
size_t rfm_assemble_ws_bytes(const rfm_layout *L);

/* Assembly of the weighted system (eq. ELMFBPINN_ls with the component-wise
 * definition of N and B): M[(r in I_j),(j,k)] = s_r * Op_r[w_j phi_jk](x_r) with the
 * partition-of-unity window w_j = what_j / sum_i what_i,
 * what_j = prod_i (1 + cos(pi (x_i - mu_ji)/hw_ji))^2 (eq. used_window_function_nd),
 * and h_r = s_r * rhs_r.  Outputs: M device [nnz] in the block layout, h device [N]. */
rfm_status rfm_assemble(const rfm_layout *L, const rfm_problem *P, double *M, double *h,
                        void *ws, size_t ws_bytes, void *stream);

/* Precision form of the assembly: the entries of rfm_assemble evaluated in binary32
 * arithmetic (inputs rounded to binary32 once; windows, features and operator in binary32)
 * and stored as binary32 (dtype RFM_F32) or as bfloat16 (RFM_BF16: round to nearest even
 * of the binary32 value, stored as its upper 16 bits).  M device [nnz] of that type in the
 * block layout; h device [N] in binary64 as in rfm_assemble; ws as rfm_assemble.  The
 * entries are not accurate enough for the filter at small tau (their error against the
 * binary64 entries is measured by the tests); they are an input for studies of the
 * precision form. */
rfm_status rfm_assemble_low(const rfm_layout *L, const rfm_problem *P, int32_t dtype, void *M,
                            double *h, void *ws, size_t ws_bytes, void *stream);

/* Bytes of device workspace rfm_rrqr_filter needs for this layout. */
size_t rfm_rrqr_ws_bytes(const rfm_layout *L);

/* sigma-RRQR filter of every block (Algorithm 1), one workgroup per block:
 * column-pivoted Householder QR (at each step the column with the largest norm
 * orthogonal to the columns already chosen, the norms recomputed exactly from the updated
 * columns; bit-equal norms go to the smallest local feature id), stopping at the first
 * step s with |R_ss| <= tau * |R_00| (threshold relative to the leading diagonal of R_j).
 * tau in [0, 1).  By default (64 < max_cols <= 512) the pivoted factorisation runs on the
 * triangular factor R0 of an unpivoted QR M_j = Q0 R0, which has the same pivots, R and
 * Q = Q0 Q1 in exact arithmetic (R-first form); rfm_rrqr_filter_tuned can select the direct
 * factorisation of M_j.  The two give the same factors up to rounding; identical columns of
 * M_j have bit-equal norms only in the direct form (the R-first form keeps one of them, as
 * rounding decides).
 * Inputs:  M device [nnz] (not modified).
 * Outputs: rank device [J]        r_j (0 <= r_j <= min(|I_j|, K_j));
 *          kept device [ncols]    kept local feature ids in pivot order, entries
 *                                 k < r_j of block j used, the rest set to -1;
 *          R    device [nrsq]     upper-triangular R_hat_j (r_j x r_j, positive
 *                                 diagonal, in the block's K_j x K_j slot; the R-first
 *                                 form also sets the rest of the slot to zero);
 *          Q    device [nnz]      explicit Q_hat_j (first r_j columns of the block's
 *                                 slot, orthonormal, Q_hat_j R_hat_j = M_j[:, kept]);
 *          ratios device [ncols]  nullable; |R_ss|/|R_00| for every step taken, the
 *                                 stopping step included, 0 elsewhere.
 * ws: device workspace of rfm_rrqr_ws_bytes(L) bytes (needed by the R-first form and the
 * persistent launch; contents on return unspecified).
 * Sizes: max_rows <= 3072 and max_cols <= 2048 (RFM_EUNSUPPORTED otherwise). */
rfm_status rfm_rrqr_filter(const rfm_layout *L, const double *M, double tau, int32_t *rank,
                           int32_t *kept, double *R, double *Q, double *ratios, void *ws,
                           size_t ws_bytes, void *stream);

/* Launch shapes of the batching form (uneven blocks).  Zero fields take the defaults. */
typedef struct {
  int32_t rrqr_threads;    /* workgroup size of the filter: 256, 512 or 1024 (1024 only for
                              blocks of at most 1024 rows); 0 = by block height */
  int32_t rrqr_persistent; /* 1: one persistent launch whose workgroups take blocks from a
                              shared counter in the given order (largest first); a form
                              of the direct factorisation (RFM_RRQR_AUTO then takes it) */
  int32_t rrqr_wgs_per_cu; /* persistent grid = rrqr_wgs_per_cu x CUs (>= 1)  */
  int32_t adj_tile;        /* columns per workgroup of the adjoint block products of LSQR
                              (a multiple of 16; 0 = about 4096 workgroups in all) */
  int32_t rrqr_algo;       /* rfm_rrqr_algo: the filter's factorisation */
} rfm_tuning;

typedef enum {
  RFM_RRQR_AUTO = 0,   /* R-first when 64 < max_cols <= 512, else direct */
  RFM_RRQR_DIRECT = 1, /* pivoted QR of M_j itself (rrqr_threads applies) */
  RFM_RRQR_RFIRST = 2  /* pivoted QR of R0 from an unpivoted QR of M_j */
} rfm_rrqr_algo;

/* Cost order of the blocks (sync, host only): block ids sorted by decreasing Householder QR
 * flops 4mnk - 2(m+n)k^2 + 4/3 k^3, k = min(m, n), ties in id order.  row_off, feat_off
 * host [J+1]; order host [J]. */
rfm_status rfm_plan_order(int32_t J, const int64_t *row_off, const int64_t *feat_off, int32_t *order);

/* rfm_rrqr_filter with an explicit block order (device [J], nullable = 0..J-1) and launch
 * shapes (nullable = defaults).  Results do not depend on either.  The persistent launch
 * needs ws (rfm_rrqr_ws_bytes). */
rfm_status rfm_rrqr_filter_tuned(const rfm_layout *L, const double *M, double tau, int32_t *rank,
                                 int32_t *kept, double *R, double *Q, double *ratios,
                                 const int32_t *order, const rfm_tuning *tune, void *ws,
                                 size_t ws_bytes, void *stream);

/* Operator of the preconditioned system M_hat S^{-1} (Proposition 3.1), or of the system
 * without the preconditioner. */
typedef enum {
  RFM_FORM_Q = 0,         /* explicit Q_hat_j: A = sum_j V_j^T Q_hat_j W_hat_j        */
  RFM_FORM_R = 1,         /* kept columns of M_j with back-substitution by R_hat_j   */
  RFM_FORM_M = 2          /* kept columns of M_j alone: A = M_hat, no preconditioner
                             (for condition estimates and comparisons; with kept = all
                             columns and rank_j = K_j it is M itself).  The stopping rule's
                             ||A|| is ||M_hat||_F, computed on the device */
} rfm_form;

typedef struct {
  int32_t form;           /* rfm_form                                       */
  const int32_t *rank;    /* device [J]                                     */
  const double *Q;        /* device [nnz]  (RFM_FORM_Q)                     */
  const double *M;        /* device [nnz]  (RFM_FORM_R, RFM_FORM_M)         */
  const int32_t *kept;    /* device [ncols] (RFM_FORM_R, RFM_FORM_M)        */
  const double *R;        /* device [nrsq] (RFM_FORM_R)                     */
  const void *Qlow;       /* device [nnz] elements of low_dtype, nullable: narrow copy of
                             Q_hat from rfm_pack_q, used by the precision form */
  int32_t low_dtype;      /* rfm_dtype of Qlow                              */
} rfm_operator;

/* Narrow copy of the explicit Q_hat for the precision form: the first r_j columns of every
 * block rounded to binary32 or bfloat16 (rfm_dtype), written in the block layout of M with
 * 4- or 2-byte elements.  Q device [nnz] binary64, Qlow device [nnz] of dtype. */
rfm_status rfm_pack_q(const rfm_layout *L, const int32_t *rank, const double *Q, int32_t dtype,
                      void *Qlow, void *stream);

/* Device time of the iteration kernels of one solve, measured with HIP events recorded
 * around each stage on the solve's stream.  Sampled: the first two iterations of every
 * batch of check_every iterations are launched eagerly with events (the rest of the batch
 * as usual, graph or eager); ms / launches is the average duration of a stage. */
typedef struct {
  double ms[5];           /* total ms of the stages: [0] forward block products (R form: with
                             the triangular solves), [1] row gather + beta, [2] adjoint block
                             products (R form: with the transposed solves), [3] alpha and the
                             rotation (R form only; the Q form does them in stage 4 and leaves
                             this 0), [4] y/w update + stop test */
  int64_t launches[5];    /* sampled launches counted (only iterations that did work) */
} rfm_kernel_times;

typedef struct {
  double atol, btol;      /* stopping tolerances (see rfm_lsqr_solve)       */
  int64_t maxit;          /* iteration limit (>= 1)                         */
  int32_t check_every;    /* iterations launched between host checks of the stop flag (>= 1) */
  int32_t use_graph;      /* 1: replay the per-check batch of launches as a HIP graph */
  rfm_kernel_times *times;/* host, nullable: sampled per-stage device times (see above) */
  double *history;        /* device, nullable, [2 * maxit]: per iteration the estimates of
                             ||r|| and ||A^T r|| (entries past the last iteration untouched;
                             plain solves only) */
  int32_t inner_dtype;    /* RFM_F64: plain LSQR.  RFM_F32 / RFM_BF16: precision form --
                             binary64 residual refinement around LSQR on the narrow copy
                             A->Qlow (products accumulated in binary32) */
  int32_t max_outer;      /* precision form: refinement steps (>= 1)        */
  int64_t max_inner;      /* precision form: iteration cap of one inner solve (>= 1) */
  double inner_tol;       /* precision form: atol = btol of the inner solves, in (0, 1) */
  int32_t adj_tile;       /* columns per workgroup of the adjoint block products (multiple of
                             16; 0 = default, see rfm_tuning) */
  double *bidiag;         /* device, nullable, [2 * maxit + 2]: the Golub-Kahan bidiagonalisation
                             A V_k = U_{k+1} B_k the solve runs on (plain solves only): entries
                             (alpha_1, beta_1) first, then after iteration i (alpha_{i+1},
                             beta_{i+1}) at [2 i], [2 i + 1]; B_k is lower bidiagonal with
                             alpha_1..alpha_k on its diagonal and beta_2..beta_{k+1} below it, and
                             its extreme singular values bound those of A from inside (entries past
                             the last iteration untouched) */
} rfm_lsqr_opts;

typedef struct {
  int64_t iters;          /* iterations performed (precision form: inner iterations in total) */
  int64_t outer;          /* precision form: refinement steps taken (0 for plain solves) */
  int64_t polish;         /* precision form: binary64 LSQR iterations of the finish (included
                             in iters)                                      */
  int32_t stop;           /* 1: S1, 2: S2, 3: maxit, 4: breakdown (exact solution) */
  int32_t warm_rejected;  /* 1: the warm start y0 was discarded (||h - A y0|| > ||h||) and the
                             solve started from 0 */
  double rnorm_est;       /* ||r|| estimate at the stop                      */
  double artnorm_est;     /* ||A^T r|| estimate at the stop                  */
  double anorm;           /* ||A|| used by the rule: sqrt(sum_j r_j)         */
  double hnorm;           /* ||h||                                           */
  double ynorm;           /* ||y|| at the stop                               */
  double relres;          /* explicit ||h - A y|| / ||h|| recomputed at the stop */
  double eta;             /* explicit ||A^T r|| / (||A|| ||r||) recomputed at the stop */
} rfm_lsqr_info;

/* Bytes of device workspace rfm_lsqr_solve needs for this layout. */
size_t rfm_lsqr_ws_bytes(const rfm_layout *L);

/* LSQR (Paige and Saunders 1982) on min ||A y - h|| with A the preconditioned operator
 * (Algorithm 2, solve step), started from y0 (nullable = 0).  Stopping rule, with the
 * fixed ||A|| = ||A||_F = sqrt(sum_j r_j):
 *   S1: ||r|| <= btol ||h|| + atol ||A|| ||y||,   S2: ||A^T r|| <= atol ||A|| ||r||,
 * on the recurrence estimates; breakdown (alpha or beta = 0) stops with the exact
 * solution.  After stopping the residuals are recomputed explicitly with the operator
 * and returned in info.
 * Precision form (opts->inner_dtype != RFM_F64): y <- y0; repeat { r = h - A y and A^T r in
 * binary64 with the full operator; stop by S1/S2 on these explicit values; first step: LSQR
 * on min ||A_low y - h|| from the current y, later steps: min ||A_low d - r|| from 0 and
 * y <- y + d, both with atol = btol = inner_tol (A_low the narrow Q_hat, binary32
 * accumulation) } while ||A^T r|| at least halves per step (and for at most max_outer
 * steps); then binary64 LSQR from y (the finish) until S1/S2.  Refinement through a
 * narrow operator converges to A_low^T (h - A y) = 0, not A^T (h - A y) = 0, which on these
 * least-squares systems (non-zero optimal residual) leaves ||A^T r|| near u_low ||A|| ||r||;
 * the finish removes that bias.  opts->maxit caps all iterations together.  With
 * inner_tol = atol = btol and max_outer = 1 the scheme is one narrow LSQR solve to the full
 * rule, the binary64 check, and a binary64 finish only where that check fails: the Krylov
 * process is never restarted, which matters on ill-conditioned systems where short inner
 * solves each lose the subspace built so far.
 * Vectors: h device [N]; y0, y device [ncols] (entry (j,k) for k < r_j at feat_off[j]+k
 * in pivot order; other entries of y are set to 0).  A warm start whose residual
 * ||h - A y0|| exceeds ||h|| is discarded and the solve starts from 0 (info->warm_rejected).  (sync): returns after the solve;
 * RFM_ENOTCONV if maxit was reached. */
rfm_status rfm_lsqr_solve(const rfm_layout *L, const rfm_operator *A, const double *h,
                          const double *y0, const rfm_lsqr_opts *opts, double *y,
                          rfm_lsqr_info *info, void *ws, size_t ws_bytes, void *stream);

/* Bytes of device workspace rfm_lsqr_multi needs for nrhs right-hand sides. */
size_t rfm_lsqr_multi_ws_bytes(const rfm_layout *L, int32_t nrhs);

/* LSQR for nrhs (1..64) right-hand sides on the same Q-form operator (sync): one Paige-Saunders
 * recurrence and stopping test (the rule of rfm_lsqr_solve, with opts->atol, btol, maxit;
 * the other options are ignored) per right-hand side, sharing every pass over Q_hat, so the
 * block products are dense matrix-matrix products.  Right-hand-side-minor layout: H device
 * [N x nrhs], Y0 (nullable) and Y device [ncols x nrhs] (entry (j,k) of right-hand side b at
 * (feat_off[j] + k) * nrhs + b).  A finished right-hand side is frozen while the others go on.
 * With Y0, each right-hand side's start passes the guard of rfm_lsqr_solve: one whose residual
 * ||h_b - A y0_b|| exceeds ||h_b|| is replaced by the zero start.
 * iters, stops, rejected (1 where the guard dropped the start): host [nrhs], nullable.
 * RFM_ENOTCONV if any right-hand side reached maxit. */
rfm_status rfm_lsqr_multi(const rfm_layout *L, const rfm_operator *A, const double *H, int32_t nrhs,
                          const double *Y0, const rfm_lsqr_opts *opts, double *Y, int64_t *iters,
                          int32_t *stops, int32_t *rejected, void *ws, size_t ws_bytes, void *stream);

/* Back-substitution a_hat_j = R_hat_j^{-1} y_j and scatter to the global coefficient
 * vector with zeros at dropped columns (Algorithm 2, output step).
 * y device [ncols] (layout of rfm_lsqr_solve), a device [ncols] (entry (j,k) at
 * feat_off[j] + k, local feature order). */
rfm_status rfm_coefficients(const rfm_layout *L, const int32_t *rank, const int32_t *kept,
                            const double *R, const double *y, double *a, void *stream);

/* Bytes of device workspace rfm_evaluate needs for a test-point layout. */
size_t rfm_evaluate_ws_bytes(const rfm_layout *L);

/* Strong rank-revealing variant of the filter (Section 2.3: the factorisation may be any
 * rank-revealing QR, strong RRQR of Gu and Eisenstat among them).  The rank r_j of every block
 * is the sigma-filter's (column-pivoted QR stopped at |R_ss| <= tau |R_00|, direct
 * factorisation); then, per block, with R = [A B; 0 C] in the current pivot order (A = R_hat),
 *   rho_iq = (A^-1 B)_iq^2 + ||C e_q||^2 ||e_i^T A^-1||^2,
 * and while max rho > f^2 the pair (i, q) of the maximum is exchanged (kept column i for
 * trailing column q; ties to the smaller i, then q) and the block refactored in its new order
 * with the same rank, at most max_rounds rounds over all blocks (each round swaps once in
 * every block that needs it; |det A| grows by more than f per swap, so the loop ends).  The
 * test runs once more after the last round: on return every block satisfies max rho <= f^2
 * unless stats[2] > 0 (max_rounds reached), and then
 * sigma_i(A) >= sigma_i(M_j) / sqrt(1 + f^2 r (n - r)) and
 * sigma_q(C) <= sigma_(r+q)(M_j) sqrt(1 + f^2 r (n - r)) (Gu and Eisenstat 1996).
 * Outputs as rfm_rrqr_filter (rank, kept in pivot order, R_hat, Q_hat; no ratios), plus
 * rho device [J]: the largest rho of the last test per block (0 where r is 0 or n_j), and
 * stats host [3]: exchanges made, rounds taken, blocks whose last test still exceeds f^2
 * (0 unless max_rounds stopped the loop).  f > 1, max_rounds >= 0 (0: the test only).
 * Sync (one host read per test).
 * ws: rfm_rrqr_strong_ws_bytes(L) device bytes.  Needs max_rows <= 3072. */
size_t rfm_rrqr_strong_ws_bytes(const rfm_layout *L);
rfm_status rfm_rrqr_strong(const rfm_layout *L, const double *M, double tau, double f, int32_t max_rounds,
                           int32_t *rank, int32_t *kept, double *R, double *Q, double *rho, int32_t *stats,
                           void *ws, size_t ws_bytes, void *stream);

/* Solution at test points and its error (Sec. 4.2 performance evaluation; eq. elm_solution
 * with the windows of eq. used_window_function_nd): u_hat(x_t) = sum over the subdomains j
 * covering x_t (strict |x - mu| < hw) of w_j(x_t) sum_k a_(j,k) Xi(w_(j,k) . (x_t - mu_j)/hw_j
 * + b_(j,k)), times the ansatz factor g(x_t) when P->ansatz is set, and, with u_exact,
 * e_L1 = mean_t |u_hat - u| / std(u) (population standard deviation over the test points).
 * Lt: a layout planned (rfm_plan) on the test points with the same subdomains and feature
 * counts; P: its x = test points [T*d] (device), mu, hw, w, b, activation as for the assembly,
 * ansatz (nullable) per test point in the assembly's layout, of which only g is read (the
 * other fields are not read).  a device [ncols] (rfm_coefficients);
 * uhat device [T]; u_exact device [T] and e_l1 host [1], both nullable together.  Sync when
 * e_l1 is requested.  ws: rfm_evaluate_ws_bytes(Lt). */
rfm_status rfm_evaluate(const rfm_layout *Lt, const rfm_problem *P, const double *a, double *uhat,
                        const double *u_exact, double *e_l1, void *ws, size_t ws_bytes, void *stream);

/* Learned warm start (the form that maps the parameters of a PDE family to LSQR starting
 * coordinates): a 3-layer perceptron n_in -> n_hidden -> n_hidden -> n_out with tanh hidden
 * layers and a linear output, binary32.  Row-major parameters on the device: W1 [n_in x H],
 * W2 [H x H], W3 [H x n_out], b1, b2 [H], b3 [n_out]; a batch of inputs X is [batch x n_in].
 * Forward: H1 = tanh(X W1 + b1), H2 = tanh(H1 W2 + b2), Y = H2 W3 + b3. */
typedef struct {
  int32_t n_in, n_hidden, n_out;
  float *W1, *b1, *W2, *b2, *W3, *b3;
} rfm_mlp;

/* Device workspace of rfm_mlp_backward for this network and batch size. */
size_t rfm_mlp_ws_bytes(const rfm_mlp *P, int32_t batch);

/* Forward pass; H1, H2 [batch x H] and Y [batch x n_out] device outputs. */
rfm_status rfm_mlp_forward(const rfm_mlp *P, const float *X, int32_t batch, float *H1, float *H2,
                           float *Y, void *stream);

/* Backward pass of the mean squared error L = sum (Y - T)^2 / (batch n_out) given the forward
 * activations: writes the parameter gradients into the buffers of G (same sizes as P), the
 * loss into *loss (device float), and uses dY [batch x n_out], dH1, dH2 [batch x H] as
 * device scratch.  Sums over the batch are taken in a fixed order. */
rfm_status rfm_mlp_backward(const rfm_mlp *P, const rfm_mlp *G, const float *X, const float *H1,
                            const float *H2, const float *Y, const float *T, int32_t batch,
                            float *dY, float *dH1, float *dH2, float *loss, void *ws,
                            size_t ws_bytes, void *stream);

/* Adam (Kingma and Ba) on n parameters: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps); step >= 1. */
rfm_status rfm_adam_step(int64_t n, float *p, const float *g, float *m, float *v, float lr,
                         float beta1, float beta2, float eps, int32_t step, void *stream);

/* out[i, :] = in[idx[i], :] for row-major [* x cols] binary32 matrices (mini-batch gather). */
rfm_status rfm_gather_rows(int32_t rows, int32_t cols, const int32_t *idx, const float *in,
                           float *out, void *stream);

/* Learned form, data and training.
 * rfm_weighted_rhs: H[r, b] = weight[r] rhs[r, b] for nrhs right-hand sides (row scaling of
 *   eq. ELMFBPINN_ls), device [N x nrhs] right-hand-side-minor.
 * rfm_solutions_to_rows: out[row0 + b, k] = (float) Y[k, b]: nrhs LSQR solutions (device
 *   [ncols x nrhs]) as rows of a binary32 target matrix [* x ncols].
 * rfm_standardize_columns: per-column mean and standard deviation over n rows (sd = 1 for a
 *   constant column), then T <- (T - mean) / sd in place; mean, sd device [cols].
 * rfm_decode_start: y0[k, b] = pred[b, k] sd[k] + mean[k] on kept coordinates, 0 elsewhere
 *   (network predictions [nrhs x ncols] to binary64 LSQR starts [ncols x nrhs]).
 * rfm_mlp_train (sync): `epochs` passes of mini-batch Adam (lr, 0.9, 0.999, 1e-8) over the n
 *   rows of X [n x n_in] and T [n x n_out]; the sample order is reshuffled every epoch
 *   (splitmix64 from `seed`, Fisher-Yates) into idx (device [n]); G, Mom, Var are gradient and
 *   moment buffers shaped like P (Mom, Var zeroed by the caller); scratch holds at least
 *   batch (n_in + 3 n_out + 4 n_hidden) + 65 floats; ws rfm_mlp_ws_bytes(P, batch) bytes;
 *   loss_history (host, nullable, [epochs]) the mean batch loss per epoch. */
rfm_status rfm_weighted_rhs(int64_t N, int32_t nrhs, const double *weight, const double *rhs, double *H,
                            void *stream);
rfm_status rfm_solutions_to_rows(int64_t ncols, int32_t nrhs, const double *Y, int64_t row0, float *out,
                                 void *stream);
rfm_status rfm_standardize_columns(int64_t n, int64_t cols, float *T, float *mean, float *sd, void *stream);
rfm_status rfm_decode_start(const rfm_layout *L, const int32_t *rank, int32_t nrhs, const float *pred,
                            const float *mean, const float *sd, double *y0, void *stream);
rfm_status rfm_mlp_train(const rfm_mlp *P, const rfm_mlp *G, const rfm_mlp *Mom, const rfm_mlp *Var,
                         const float *X, const float *T, int64_t n, int32_t batch, int32_t epochs, float lr,
                         uint64_t seed, int32_t *idx, float *scratch, size_t scratch_floats, void *ws,
                         size_t ws_bytes, float *loss_history, void *stream);

/* Autotuner of the batching form (sync).  Times, with HIP events on `stream`, every
 * candidate launch shape of the filter on the caller's data (the R-first form when
 * max_cols <= 512, and the direct form with rrqr_threads in {256, 512, 1024} as default
 * and persistent launches with 1 or 2 workgroups per CU) and then the adjoint tile
 * of LSQR (adj_tile in {16, 32, 64, 128, 256}) over a short solve of lsqr_iters iterations
 * on h, and writes the fastest shapes to *best.  The filter outputs (rank, kept, R, Q,
 * ratios) hold the result of the winning filter shape.
 * ms_out / cand_out (host, nullable, capacity 32) receive every candidate's time and shape;
 * *ncand their number.  ws: max(rfm_rrqr_ws_bytes, rfm_lsqr_ws_bytes) bytes of device memory;
 * y_scratch: device [ncols]. */
rfm_status rfm_autotune(const rfm_layout *L, const double *M, double tau, int32_t *rank,
                        int32_t *kept, double *R, double *Q, double *ratios, const int32_t *order,
                        const double *h, int64_t lsqr_iters, double *y_scratch, void *ws,
                        size_t ws_bytes, rfm_tuning *best, double *ms_out, rfm_tuning *cand_out,
                        int32_t *ncand, void *stream);

/* Description of the last failure on the calling thread ("" if none). */
const char *rfm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RFM_H */
