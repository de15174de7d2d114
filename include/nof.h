/*
 * nof.h -- C ABI of the MI355X (gfx950) density-fitted JK / generalized-Fock
 * library, the per-iteration hot path of natural-orbital-functional (NOF)
 * orbital optimisation (DoNOF 2.0, arXiv 2512.13550).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Array arguments are DEVICE pointers (HBM), row-major, owned by the
 *    caller.  The library never allocates or frees caller memory; scratch
 *    space is passed in as a caller-owned workspace whose size the matching
 *    *_ws() query returns.
 *  - Work is enqueued asynchronously on `stream` (0 = the null stream).
 *    Scalar results are written to device memory.
 *  - Return value: NOF_OK (0) or a negative nof_status.  All shape, pointer,
 *    dtype, precision and workspace checks run on the host before anything is
 *    launched; on failure nothing is enqueued.  A failed launch returns
 *    NOF_E_HIP.  Faults inside a kernel surface at the caller's next
 *    synchronisation, as for any HIP work.
 *  - No C++ exception crosses this boundary.
 *  - Entry points are re-entrant; calls on different streams may overlap as
 *    long as they do not share output or workspace buffers.
 *
 * Notation (paper, Theory and NO Optimization sections):
 *   naux   auxiliary (density-fitting) basis size, index P
 *   nbf    AO basis size, indices mu, nu
 *   norb   number of natural orbitals, indices p, q, r, s
 *   B[P][mu][nu]  RI three-index tensor (ERITYP='RI'), symmetric in (mu,nu)
 *   C[mu][p]      NO coefficients, column p = orbital p
 *   b[P][p][q]    = (C^T B^P C)_pq, symmetric in (p,q)
 *   D[P][p]       = b^P_pp
 *   J_pq = sum_P D[P][p] D[P][q]      Coulomb integrals (pp|qq)
 *   K_pq = sum_P (b^P_pq)^2            exchange integrals (pq|qp)
 *   Eq. (PNOF): E = 2 sum_p n_p h_pp + sum_pq cJ_pq J_pq - sum_pq cK_pq K_pq
 *     with cJ = A and cK = B + C (L = K for real orbitals).
 */
#ifndef NOF_H
#define NOF_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NOF_OK = 0,
  NOF_E_NULL = -1,          /* a required pointer is NULL                        */
  NOF_E_DIM = -2,           /* a size is out of range or inconsistent            */
  NOF_E_DTYPE = -3,         /* unsupported storage type for this argument        */
  NOF_E_PREC = -4,          /* unsupported precision mode for this entry point   */
  NOF_E_WORKSPACE = -5,     /* workspace NULL or smaller than the *_ws() query   */
  NOF_E_HIP = -6,           /* a HIP runtime call or kernel launch failed        */
  NOF_E_NOT_CONVERGED = -7, /* iteration cap reached before the tolerance        */
  NOF_E_ARG = -8,           /* an argument value is invalid (e.g. a handle)      */
  NOF_E_INTERNAL = -99
} nof_status;

/* Storage type of a large tensor argument (B, b).
 *   NOF_BF16X4  B as the four fixed-point BF16 planes written by nof_split_B
 *               (NOF_P_BF16X10 only).
 *   NOF_I8X4    B as the four fixed-point INT8 planes and row exponents
 *               written by nof_split_B_i8 (NOF_P_I8X10 only). */
typedef enum { NOF_F64 = 0, NOF_F32 = 1, NOF_BF16 = 2, NOF_BF16X4 = 3, NOF_I8X4 = 4 } nof_dtype;

/* Arithmetic used by the matrix-core (MFMA) contractions.
 *   NOF_P_F64     FP64 MFMA, FP64 accumulation.
 *   NOF_P_F32     FP32 MFMA, FP32 accumulation inside one auxiliary slab,
 *                 FP64 across slabs.
 *   NOF_P_BF16X1  one BF16 product, FP32 accumulation.
 *   NOF_P_BF16X3  operands split into BF16 hi+lo, products hi*hi+hi*lo+lo*hi.
 *   NOF_P_BF16X6  operands split into BF16 hi+mid+lo, the six products whose
 *                 combined order of magnitude is at most two splits down;
 *                 every 32-deep stage is added into FP64 accumulators.  The
 *                 exchange-type Fock term is the x10 one below.
 *   NOF_P_BF16X10 fixed-point split (Ozaki-type error-free split on BF16):
 *                 every row of X and column of Y gets one grid over the whole
 *                 contraction, 2^E above its largest magnitude, and four BF16
 *                 pieces x = sum_{q<4} n_q 2^(E-7-8q) + r, integers
 *                 |n_q| <= 128, |r| <= 2^(E-32); the ten products of order
 *                 <= 3.  The order-0 products are integers of at most 2^14
 *                 units, so their FP32 running sum is exact for up to 1024
 *                 terms; longer contractions add it to FP64 every 1024 terms.
 *                 Orders 1..3 share a second FP32 accumulator.  T and b are
 *                 stored in FP32.  The exchange-type Fock term uses three
 *                 element-wise pieces (six products) instead.
 *   NOF_P_I8X10   the fixed-point split with INT8 pieces on the INT8 matrix
 *                 cores (nof_mo_transform with B from nof_split_B_i8, and the
 *                 exchange-type Fock term): one grid per row / column, 2^E the
 *                 smallest power of two with max|x| 2^(7-E) < 127.5,
 *                 x = n_0 2^(E-7) + sum_{q=1..3} n_q 2^(E-7-7q) + r,
 *                 |n_0| <= 127, |n_q| <= 64, |r| <= 2^(E-29); the ten
 *                 products of order <= 3 in four int32 accumulators (one per
 *                 order; exact for contractions shorter than 65536), combined
 *                 exactly in FP64.  T and b stored in FP32.  The exchange-type
 *                 term (Naux <= 65536) goes through the symmetric per-q
 *                 products G^q_rs = sum_P b^P_qr b^P_qs (see nof_gen_fock):
 *                 one INT8 contraction over P per q with one grid per (q, r)
 *                 over all slabs, exact int32 sums written in FP64, chunks of
 *                 q whose planes and G fit 4 GiB of workspace, then the
 *                 cK-weighted sum over q in FP64.  Beyond Naux = 65536 it sums
 *                 groups of auxiliary slabs as one INT8 contraction each (as
 *                 many slabs as keep slabs x 64-padded rows within 65536), one
 *                 grid per row of b^P and of cK o b^P over the group, an FP64
 *                 partial per group, in chunks whose planes fit 8 GiB.  The
 *                 batched plan takes that term as in NOF_P_BF16X10.
 * Reductions that produce J, K, lambda, g and E always accumulate in FP64. */
typedef enum {
  NOF_P_F64 = 0, NOF_P_F32 = 1, NOF_P_BF16X1 = 2, NOF_P_BF16X3 = 3, NOF_P_BF16X6 = 4,
  NOF_P_BF16X10 = 5, NOF_P_I8X10 = 6
} nof_prec;

/* Human-readable text for a status code (static storage, never NULL). */
const char* nof_status_str(int status);

/* ---------------------------------------------------------------------------
 * Fixed-point split of the three-index tensor for NOF_P_BF16X10, done once
 * per B (every orbital iteration reuses B; Single Point Energy Calculations,
 * ERITYP='RI').  Row (P, mu) of B^P gets one grid over its whole length:
 * with 2^E above the row's largest |value|, each value becomes
 *   v = sum_{q<4} n_q 2^(E-7-8q) + r,  n_q integers (exact in BF16),
 *   |n_q| <= 128, |r| <= 2^(E-32).
 * B       [naux][nbf][nbf] FP64 or FP32 (Bt), symmetric, device.
 * planes  out, at least nof_split_B_bytes(naux, nbf) bytes, device (caller
 *         owned); layout [4][naux][nbf][ldk], ldk = nbf rounded up to a
 *         multiple of 32, zero for nu >= nbf.  Pass it as B with
 *         Bt = NOF_BF16X4 to nof_mo_transform / nof_mo_transform_stage1.
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_DTYPE (Bt not F64/F32),
 *         NOF_E_WORKSPACE (planes_bytes too small), NOF_E_HIP.
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * The same once-per-B split with INT8 pieces for NOF_P_I8X10: row (P, mu)
 * of B^P gets the grid exponent E of NOF_P_I8X10 above and four INT8 pieces.
 * B       [naux][nbf][nbf] FP64 or FP32 (Bt), symmetric, device.
 * out     at least nof_split_B_i8_bytes(naux, nbf) bytes, device (caller
 *         owned): planes [4][naux][nbf][ldk] (int8, ldk = nbf rounded up to
 *         a multiple of 64, zero for nu >= nbf), then at the next 256-byte
 *         boundary the exponents [naux][nbf] (int32).  Pass it as B with
 *         Bt = NOF_I8X4 to nof_mo_transform.
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_DTYPE (Bt not F64/F32),
 *         NOF_E_WORKSPACE (out_bytes too small), NOF_E_HIP.
 * ------------------------------------------------------------------------- */
size_t nof_split_B_i8_bytes(int naux, int nbf);
int nof_split_B_i8(int naux, int nbf, const void* B, int Bt, void* out, size_t out_bytes,
                   hipStream_t stream);

size_t nof_split_B_bytes(int naux, int nbf);
int nof_split_B(int naux, int nbf, const void* B, int Bt, void* planes, size_t planes_bytes,
                hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Orbital transformation (Single Point Energy Calculations, ERITYP='RI':
 * the RI route whose transformation is fourth order).
 *
 *   b^P = C^T B^P C  for P = 0..naux-1,   D[P][p] = b^P_pp.
 *
 * B   [naux][nbf][nbf], storage Bt.  Must be symmetric in (mu,nu): the
 *     kernel reads B^P_{nu mu} where the definition has B^P_{mu nu}.
 * C   [nbf][norb] FP64 (the master copy; converted or split on load).
 * b   out [naux][norb][norb], storage bt; written exactly symmetric.
 * D   out [naux][norb] FP64, may be NULL.
 * prec / storage:
 *     NOF_P_F64            Bt = bt = NOF_F64
 *     NOF_P_F32            Bt = bt = NOF_F32
 *     NOF_P_BF16X1..X10    Bt = NOF_F32 (or NOF_BF16 with X3/X6, or
 *                          NOF_BF16X4 with X10), bt = NOF_F32;
 *                          B and T are split into BF16 pieces in the loaders
 *                          (B not at all when given as NOF_BF16X4 planes),
 *                          C once per call (three pieces for a BF16-stored B,
 *                          four with X10).
 *     NOF_P_I8X10          Bt = NOF_I8X4 (nof_split_B_i8), bt = NOF_F32; C
 *                          split once per call, B^P C split by a pass (one
 *                          grid per column of each B^P C) between the stages.
 * ws  workspace of at least nof_mo_transform_ws(...) bytes (holds B^P C and
 *     the BF16 pieces of C; with X10 also the column maxima of B^P C that the
 *     first stage writes as it stores them, which give the second stage the
 *     grids of its split without another pass over B^P C; with I8X10 the
 *     INT8 planes of C, those maxima and the INT8 planes of B^P C).
 *
 * With naux = 1 and B = H (the AO one-electron matrix) this yields
 * h = C^T H C, the one-electron integrals of Eq. (Energy) in the NO basis.
 * ------------------------------------------------------------------------- */
size_t nof_mo_transform_ws(int naux, int nbf, int norb, int Bt, int bt, int prec);
int nof_mo_transform(int naux, int nbf, int norb,
                     const void* B, int Bt, const double* C,
                     void* b, int bt, double* D,
                     int prec, void* ws, size_t ws_bytes, hipStream_t stream);

/* The two stages of nof_mo_transform as separate calls (same arguments and
 * rules; not for NOF_P_I8X10, whose second stage takes the first stage's
 * column maxima: NOF_E_PREC), for callers that keep the half-transformed
 * tensor or time the stages:
 *   stage 1:  T[P][mu][q] = (B^P C)_{mu q}        T: [naux][nbf][norb], storage Tt
 *   stage 2:  b^P = C^T T^P, D[P][p] = b^P_pp     (exactly symmetric b)
 * Tt is the storage of b for the precision mode.  ws (at least
 * nof_mo_transform_stage_ws() bytes) holds the BF16 pieces of C in the split
 * forms (and, for X10, the grid exponents of the operand split in the
 * loader: rows of an FP32 B, columns of T); FP64/FP32 ignore it (it may be
 * NULL).  The stages share nothing through ws. */
size_t nof_mo_transform_stage_ws(int naux, int nbf, int norb, int prec);
int nof_mo_transform_stage1(int naux, int nbf, int norb, const void* B, int Bt,
                            const double* C, void* T, int Tt, int prec,
                            void* ws, size_t ws_bytes, hipStream_t stream);
int nof_mo_transform_stage2(int naux, int nbf, int norb, const void* T, int Tt,
                            const double* C, void* b, int bt, double* D, int prec,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Coulomb and exchange integrals in the NO basis (Eq. PNOF's J and K).
 *
 *   J = D^T D            (J_pq = (pp|qq)),   may be NULL to skip
 *   K_pq = sum_P b_pq^2  (K_pq = (pq|qp)),   may be NULL to skip
 *
 * b   [naux][norb][norb] storage bt (NOF_F64 or NOF_F32), symmetric.  Only
 *     the upper triangle (p <= q) is read for K.
 * D   [naux][norb] FP64.
 * J,K out [norb][norb] FP64, exactly symmetric.  Accumulation is FP64 in a
 *     fixed order, so results repeat bit for bit.
 * ------------------------------------------------------------------------- */
size_t nof_jk_diag_ws(int naux, int norb, int bt);
int nof_jk_diag(int naux, int norb, const void* b, int bt, const double* D,
                double* J, double* K, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Generalized-Fock (Lagrangian) build and orbital gradient (NO Optimization:
 * the Lagrangian with multipliers lambda, and g_pq = dE/dy_pq =
 * 4(lambda_pq - lambda_qp) for the rotation C <- C exp(y)).
 *
 * With W = D cJ:
 *   lambda_rs = n_s h_rs + sum_P b^P_rs W[P][s]
 *               - sum_P sum_q b^P_rq cK_sq b^P_qs
 *   grad = 4 (lambda - lambda^T)
 *
 * n       [norb] occupation numbers (0 <= n <= 1), FP64.
 * h       [norb][norb] FP64, h = C^T H C.
 * cJ, cK  [norb][norb] FP64, must be symmetric (Eq. PNOF coefficients).
 * lambda  out [norb][norb] FP64.          grad  out, may be NULL.
 * K_opt   if not NULL, also receives K (same definition as nof_jk_diag),
 *         from one pass over the upper half of b.
 * prec    NOF_P_F64 (bt = NOF_F64), NOF_P_F32 or a split form (bt = NOF_F32)
 *         for the matrix-core contraction (X6 and X10: three element-wise
 *         BF16 pieces, FP32 accumulation over 64 q of a slab, FP64 beyond; I8X10:
 *         the symmetric per-q products below as INT8 fixed-point
 *         contractions over P, exact int32 sums, FP64 beyond).
 * FP64, FP32 and I8X10: b^P is symmetric, so the exchange-type sum is
 *   sum_q cK_sq G^q_rs,   G^q_rs = sum_P b^P_qr b^P_qs,
 * and every G^q is symmetric in (r, s): the matrix cores form the upper
 * tiles of the G^q (Naux Norb^2 (Norb+1) multiply-adds, half those of the
 * product over (P, q)), at most 4 GiB of them at a time in the workspace,
 * and a pass adds cK_sq G^q_rs over q in a fixed order; the Coulomb-type sum
 * comes from the pass over the upper half of b (with K); FP32 b: FP32
 * products and sums over P, G in FP64.  The x1 / x3 forms: the two sums over
 * P are one contraction (nof_fock_terms),
 * the Coulomb-type sum being the exchange-type one with cK_sq b^P_qs
 * replaced by -W[P][s] on q = s, applied to the right operand as it is
 * staged.
 * ------------------------------------------------------------------------- */
size_t nof_gen_fock_ws(int naux, int norb, int bt, int prec);
int nof_gen_fock(int naux, int norb, const void* b, int bt, const double* D,
                 const double* n, const double* h,
                 const double* cJ, const double* cK,
                 double* lambda, double* grad, double* K_opt,
                 int prec, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Both Fock terms of lambda (NO Optimization), as nof_gen_fock computes them
 * (x1, x3: in one matrix-core contraction; FP64, FP32 and the other forms:
 * the exchange-type term minus the Coulomb-type term of the pass):
 *   W = D cJ,
 *   F_rs = F2_rs - F1_rs = sum_P sum_q b^P_rq (cK_sq b^P_qs - [q = s] W[P][s])
 * so that lambda_rs = n_s h_rs - F_rs (nof_lambda_grad with F1 = NULL).
 * b, bt, D, cJ, cK, prec as in nof_gen_fock.  F out [norb][norb] FP64 (not
 * symmetric).  ws: at least nof_fock_terms_ws(naux, norb, bt, prec) bytes.
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_DTYPE, NOF_E_PREC, NOF_E_WORKSPACE,
 * NOF_E_HIP.
 * ------------------------------------------------------------------------- */
size_t nof_fock_terms_ws(int naux, int norb, int bt, int prec);
int nof_fock_terms(int naux, int norb, const void* b, int bt, const double* D, const double* cJ,
                   const double* cK, double* F, int prec, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The exchange-type term of the generalized Fock build alone (the last sum
 * of lambda above, NO Optimization), as nof_gen_fock computes it:
 *   F2_rs = sum_P sum_q b^P_rq cK_sq b^P_qs
 * b, bt, cK, prec as in nof_gen_fock.  F2 out [norb][norb] FP64 (not
 * symmetric).  ws: at least nof_exchange_fock_ws(...) bytes.
 * ------------------------------------------------------------------------- */
size_t nof_exchange_fock_ws(int naux, int norb, int bt, int prec);
int nof_exchange_fock(int naux, int norb, const void* b, int bt, const double* cK, double* F2,
                      int prec, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The Coulomb-type term of the generalized Fock build alone (the middle sum
 * of lambda above, NO Optimization), with K from the same pass over the
 * upper half of b (an HBM-bound pass; with the x1 and x3 forms nof_gen_fock
 * folds this term into the exchange-type contraction instead):
 *   W = D cJ,   F1_rs = sum_P b^P_rs W[P][s],   K_pq = sum_P (b^P_pq)^2
 * b, bt, D, cJ as in nof_gen_fock.  F1 out [norb][norb] FP64 (not symmetric);
 * K_opt out [norb][norb] FP64 or NULL.  FP64 accumulation in a fixed order.
 * ws: at least nof_coulomb_fock_ws(naux, norb, bt) bytes.
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_DTYPE, NOF_E_WORKSPACE, NOF_E_HIP.
 * ------------------------------------------------------------------------- */
size_t nof_coulomb_fock_ws(int naux, int norb, int bt);
int nof_coulomb_fock(int naux, int norb, const void* b, int bt, const double* D, const double* cJ,
                     double* F1, double* K_opt, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Lagrange multipliers and orbital gradient from the two Fock terms (NO
 * Optimization): lambda_rs = n_s h_rs + F1_rs - F2_rs, grad = 4(lambda -
 * lambda^T), as nof_gen_fock forms them.  n [norb], h, F1, F2 [norb][norb]
 * FP64 device; F1 may be NULL, then F2 is the combined F2 - F1 of
 * nof_fock_terms; lambda out [norb][norb]; grad out or NULL.  No workspace.
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_HIP.
 * ------------------------------------------------------------------------- */
int nof_lambda_grad(int norb, const double* n, const double* h, const double* F1, const double* F2,
                    double* lambda, double* grad, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Energy of Eq. (PNOF):
 *   E = 2 sum_p n_p h_pp + sum_pq cJ_pq J_pq - sum_pq cK_pq K_pq
 * All inputs [norb] or [norb][norb] FP64; E is one FP64 device scalar.
 * Deterministic fixed-order FP64 reduction: fixed chunks summed by many
 * workgroups into ws, then the partials in a fixed tree.
 * ws  at least nof_energy_ws(norb) bytes (the partial sums).
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_WORKSPACE, NOF_E_HIP.
 * ------------------------------------------------------------------------- */
size_t nof_energy_ws(int norb);
int nof_energy(int norb, const double* n, const double* h,
               const double* J, const double* K,
               const double* cJ, const double* cK, double* E, void* ws, size_t ws_bytes,
               hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Coefficients of Eq. (PNOF) from the cumulant matrices of the (2,2)-positivity
 * reconstruction (Theory: cumulant blocks lambda^{sigma sigma} and
 * lambda^{alpha beta} in terms of Delta and Pi):
 *   cJ = 2 (n n^T - Delta),   cK = n n^T - Delta - Pi
 * n [norb]; Delta, Pi, cJ, cK [norb][norb], all FP64.
 * ------------------------------------------------------------------------- */
int nof_coeffs_from_cumulant(int norb, const double* n, const double* Delta,
                             const double* Pi, double* cJ, double* cK,
                             hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Orbital-rotation step, FP64 (NO Optimization: the NOs are updated by a
 * unitary transformation U = exp(y) of an antisymmetric y; orbitals are the
 * columns of C, so C <- C U; y comes from ADAM on the orbital gradient).
 *
 * nof_expm_antisym: U = exp(y), y [norb][norb] antisymmetric FP64.  Scaling
 *   and squaring with a degree-12 Taylor polynomial; the scaling power is
 *   chosen on the device (||y/2^s||_F <= 1/4, s <= 16), so the call never
 *   synchronises.  Accuracy is about 1e-15 for ||y||_F <= 2^14.
 * nof_rotate_orbitals: Cout = C U, C and Cout [nbf][norb] (must not alias),
 *   U [norb][norb]; ws of nof_rotate_orbitals_ws() bytes.
 * nof_adam_step: element-wise ADAM (Kingma and Ba) on the gradient g:
 *   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   y = -lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),
 *   t >= 1 is the step counter.  For antisymmetric g, y is exactly
 *   antisymmetric.  m, v [norb][norb] are caller-owned state (zero at t = 1).
 * ------------------------------------------------------------------------- */
size_t nof_expm_antisym_ws(int norb);
int nof_expm_antisym(int norb, const double* y, double* U, void* ws, size_t ws_bytes,
                     hipStream_t stream);
size_t nof_rotate_orbitals_ws(int nbf, int norb);
int nof_rotate_orbitals(int nbf, int norb, const double* C, const double* U, double* Cout,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* Orthonormality check and repair of the NOs (Natural Orbital Optimization:
 * the orbitals are orthonormal, the constraint whose multipliers are lambda;
 * products of rotations keep it only up to rounding).
 *   E = C^T S C - I,  err = max_pq |E_pq|  (a non-finite entry counts as +inf)
 *   if err > tol:  C <- C (I - E/2)
 * one Newton-Schulz step of the polar decomposition, after which the error is
 * -3/4 E^2 + 1/4 E^3 (of order err^2).
 * C    [nbf][norb] FP64, device, in/out (unchanged when err <= tol).
 * S    [nbf][nbf] FP64 AO overlap, device, or NULL for an orthonormal AO basis.
 * tol  >= 0 (else NOF_E_ARG).
 * err  device FP64 scalar, out, may be NULL.
 * ws   at least nof_orthonormalize_ws(nbf, norb) bytes.  Nothing is read back:
 *      the repair runs predicated on the device-side check.
 * Errors: NOF_E_DIM, NOF_E_NULL (C), NOF_E_ARG, NOF_E_WORKSPACE, NOF_E_HIP. */
size_t nof_orthonormalize_ws(int nbf, int norb);
int nof_orthonormalize(int nbf, int norb, double* C, const double* S, double tol, double* err,
                       void* ws, size_t ws_bytes, hipStream_t stream);

int nof_adam_step(int norb, const double* g, double* m, double* v, int t, double lr,
                  double beta1, double beta2, double eps, double* y, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * One step of the iterative diagonalization of the generalized pseudo-
 * Fockian (NO Optimization: the alternative to orbital rotations selected by
 * IORBOPT = 1; lambda is symmetric at the minimum, so a symmetric matrix
 * whose off-diagonal elements are lambda's asymmetry is diagonal there).
 *
 *   F_pq = F_qp = clamp(s_pq (lambda_qp - lambda_pq), -maxoff, maxoff),
 *   s_pq = +1 if diag_p <= diag_q else -1 (p < q),   F_pp = diag_p,
 *
 * (the orientation makes the first-order rotation a descent step for every
 * pair; the paper leaves the diagonal open).  F is diagonalized (cyclic
 * Jacobi, rotations of at most pi/4); eigenvectors are matched to orbitals
 * greedily by overlap (the largest |U_rk| of a still-free orbital r and
 * eigenvector k first; ties to the smaller r, then k), each with a
 * non-negative component on its orbital: V[:, r] is that eigenvector and
 * eig[r] its eigenvalue.  The caller
 * then forms C <- C V (nof_rotate_orbitals) and passes eig as the next
 * step's diag.
 *
 * lambda  [norb][norb] FP64 device.   diag  [norb] FP64 device, or NULL for
 *         lambda_pp (the first step of a run).   maxoff > 0.
 * V       out [norb][norb] FP64.      eig   out [norb] FP64 or NULL.
 * info    device int[2] or NULL: [0] Jacobi sweeps (-1: not converged),
 *         [1] rounds of the matching (each takes at least one pair).
 * ws      nof_pseudo_fock_diag_ws(norb) bytes.  norb <= 65536.
 * Synchronises the stream once per Jacobi sweep (not capturable).
 * Errors: NOF_E_DIM, NOF_E_NULL, NOF_E_ARG (maxoff, or lambda not finite),
 * NOF_E_WORKSPACE, NOF_E_HIP, NOF_E_NOT_CONVERGED (40 sweeps; outputs are
 * written from the last sweep).
 * ------------------------------------------------------------------------- */
size_t nof_pseudo_fock_diag_ws(int norb);
int nof_pseudo_fock_diag(int norb, const double* lambda, const double* diag, double maxoff,
                         double* V, double* eig, int* info, void* ws, size_t ws_bytes,
                         hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Occupation-number update at fixed orbitals, FP64 (Occupation Number
 * Optimization; orbital-pairing structure of Eq. OmegaG and sum rule Eq. sum1).
 *
 * members  [ns][ng+1] int, device: subspace g lists its strongly occupied
 *          orbital first, then its ng weak orbitals (distinct, < norb).
 *          Orbitals in no subspace have n = 0.  Out-of-range entries are
 *          detected on the device: info[2] = NOF_E_ARG and nothing else is
 *          written.
 * map      NOF_MAP_TRIG: n_g = (1 + cos^2 x_g)/2, n_{p_i} = h_g prod_{j<i}
 *          cos^2 x_j sin^2 x_i, the last weak orbital takes the rest;
 *          NOF_MAP_SOFTMAX: n_g = 1/(1 + sum_k e^{x_k}), n_{p_i} = n_g e^{x_i},
 *          evaluated with numerator and denominator scaled by e^{-m},
 *          m = max(0, max_k x_k), so it is finite for every x.
 * gamma    [ns][ng] variables (trig: x_g then x_1..x_{ng-1}; softmax x_1..x_ng).
 * func     NOF_FUNC_HF (Delta = Pi = 0), NOF_FUNC_PNOF5 (independent pairs:
 *          Delta_pq = n_p n_q and Pi_pq = -+sqrt(n_p n_q) within a subspace,
 *          Pi_pp = n_p; see nof_functional_coeffs) or NOF_FUNC_PNOF7 (PNOF5
 *          within each subspace; between orbitals of different subspaces
 *          Delta_pq = 0 and Pi_pq = -Phi_p Phi_q, Phi_p = sqrt(n_p (1 - n_p)):
 *          the interpair static term of Table 1's PNOF7, cited by the paper).
 * hdiag    h_pp = hdiag[p * hstride] (hstride = norb + 1 reads the diagonal of
 *          a full h).  J, K [norb][norb] FP64.
 * E = 2 sum_p n_p h_pp + sum_pq cJ(n)_pq J_pq - sum_pq cK(n)_pq K_pq.
 *
 * nof_occ_energy_grad: n [norb], E (scalar), dEdgamma [ns][ng]; any output may
 *   be NULL.
 * nof_occ_optimize: L-BFGS (memory 8, two-loop recursion, Armijo backtracking
 *   from step 1, initial step 0.1/max|pg|) on gamma in place, in one
 *   workgroup with no host round trip.  Trig variables are kept in the box
 *   [1e-12, pi/2 - 1e-12]: the map is even and pi-periodic in every angle,
 *   so the box reaches every occupation vector, and E's kinks in the angles
 *   (a weak occupation reaching 0, where PNOF5's sqrt(n_p n_q) terms are not
 *   differentiable) lie on its faces.  The start is projected onto the box,
 *   trial points are projected, the direction is zero on variables held at a
 *   face, and pg is the projected gradient (components pushing out through a
 *   face a variable sits on are 0).  Softmax variables are unbounded (pg = g).
 *   Stops when max|pg| <= tol, or when max|pg| <= 1e-5 and two consecutive
 *   steps change E by at most 1e-14 max(1,|E|), or after maxit iterations.
 *   info[0] = iterations, info[1] = 1 if converged, info[2] = 0 or a
 *   device-detected status.
 * nof_functional_coeffs: cJ = 2(nn^T - Delta), cK = nn^T - Delta - Pi for
 *   the functional (Eq. PNOF coefficients for the NO step); info may be NULL.
 * ws: nof_occ_ws() bytes (all three calls).
 * ------------------------------------------------------------------------- */
typedef enum { NOF_MAP_TRIG = 0, NOF_MAP_SOFTMAX = 1 } nof_map;
typedef enum { NOF_FUNC_HF = 0, NOF_FUNC_PNOF5 = 1, NOF_FUNC_PNOF7 = 2 } nof_functional;
size_t nof_occ_ws(int norb, int ns, int ng);
int nof_occ_energy_grad(int norb, int ns, int ng, const int* members, int map, int func,
                        const double* gamma, const double* hdiag, int hstride,
                        const double* J, const double* K, double* n, double* E,
                        double* dEdgamma, int* info, void* ws, size_t ws_bytes,
                        hipStream_t stream);
int nof_occ_optimize(int norb, int ns, int ng, const int* members, int map, int func,
                     const double* hdiag, int hstride, const double* J, const double* K,
                     double* gamma, double* n, double* E, int* info, int maxit, double tol,
                     void* ws, size_t ws_bytes, hipStream_t stream);
/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): nof_occ_optimize with its scratch in a static device array of
 * 32 MiB per GPU (allocated with the library's code object on each GPU it
 * runs on, held until the process ends).  Same arguments and results as
 * nof_occ_optimize without ws/ws_bytes; problems whose nof_occ_ws(norb, ns,
 * ng) exceeds 32 MiB (about norb > 2000) return NOF_E_DIM.  Uses the scratch
 * of the current device: stream must belong to it.  Every call on a GPU
 * shares that GPU's scratch, so calls that overlap on one GPU (other streams
 * or threads) race; every call writes all scratch it reads, so nothing must
 * start at zero.  Allocates nothing. */
int nof_occ_optimize_noalloc(int norb, int ns, int ng, const int* members, int map, int func,
                             const double* hdiag, int hstride, const double* J, const double* K,
                             double* gamma, double* n, double* E, int* info, int maxit,
                             double tol, hipStream_t stream);
int nof_functional_coeffs(int norb, int ns, int ng, const int* members, int func,
                          const double* n, double* cJ, double* cK, int* info, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched form: ninst instances sharing one B (for example the finite-field
 * instances H_i = H + F_i d of the nonlinear-optical-properties workflow),
 * each with its own C_i, H_i, occupations and coefficients.  One iteration
 * produces, for every instance, the same lambda_i, g_i and E_i as
 * nof_mo_transform + nof_jk_diag + nof_gen_fock + nof_energy would, but B is
 * read once for all instances (their C_i are packed side by side) and every
 * later step is a single instance-batched launch.
 *
 *   B      [naux][nbf][nbf], storage NOF_F64 (prec NOF_P_F64) or NOF_F32
 *          (prec NOF_P_F32: FP32 matrix-core products, FP64 reductions), or
 *          the fixed-point planes of nof_split_B (prec NOF_P_BF16X10: the x10
 *          transform and exchange-type term of nof_mo_transform and
 *          nof_gen_fock: one first-stage launch over the packed columns, the
 *          second stage and the exchange-type term of all instances in one
 *          launch each; ninst * norb <= 2^20)
 *   C      [ninst][nbf][norb]     H  [ninst][nbf][nbf]    n  [ninst][norb]
 *   cJ, cK [ninst][norb][norb] (symmetric)
 *   E      out [ninst]      lambda, grad  out [ninst][norb][norb] (grad may be NULL)
 *   ws     nof_plan_ws(plan) bytes; it also holds b_i, J_i, K_i between calls.
 *
 * nof_plan_create / nof_plan_destroy: host object holding sizes, the tuned
 *   configuration and, once captured, a HIP graph of one iteration.
 * nof_plan_autotune: runs one iteration, then times each candidate workgroup
 *   tile (128 or 64) of the two transform stages and the exchange-type
 *   contraction, and its split over P, keeping the fastest (NOF_P_I8X10:
 *   its INT8 transform stages have one tile shape, 128; the stage tiles are
 *   ignored); finishes with one iteration in the chosen configuration.  The
 *   fixed-point forms sum every output element in the same order at either
 *   tile edge, so their results do not depend on the tiles (only on the
 *   split).  Synchronises `stream`.
 * nof_plan_get_config / nof_plan_set_config: int[4] = {tile stage 1, tile
 *   stage 2, tile exchange, P-split count of the exchange term}, so a caller
 *   can cache a tuning result.
 * nof_plan_capture: records one iteration on `stream` (not the null stream)
 *   into a graph bound to these exact pointers; nof_plan_launch replays it
 *   (one hipGraphLaunch), reading the current contents of the inputs.
 * ------------------------------------------------------------------------- */
typedef struct nof_plan_s* nof_plan;
int nof_plan_create(nof_plan* plan, int ninst, int naux, int nbf, int norb, int prec);
/* Workspace layout of a plan (host only, no GPU work): the byte offset and
 * size of each of its regions, in order (first min(count, max_regions)
 * entries; offsets or bytes may be NULL).  Returns the region count, or
 * NOF_E_NULL / NOF_E_ARG.  Regions are 256-byte aligned, disjoint and end
 * within nof_plan_ws(plan); the order is: packed C, T, b, D, the one-electron
 * half transform, h, J, K, W, K partials, F1 partials, F2 partials, F1, F2,
 * energy partials, and for NOF_P_BF16X10 the planes of the packed C, the
 * column maxima of T per row tile, the grid exponents of T's columns and
 * every instance's cK transposed in FP32 (size 0 otherwise). */
int nof_plan_layout(nof_plan plan, size_t* offsets, size_t* bytes, int max_regions);
size_t nof_plan_ws(nof_plan plan);
int nof_plan_get_config(nof_plan plan, int* cfg);
int nof_plan_set_config(nof_plan plan, const int* cfg);
int nof_plan_iteration(nof_plan plan, const void* B, const double* C, const double* H,
                       const double* n, const double* cJ, const double* cK, double* E,
                       double* lambda, double* grad, void* ws, size_t ws_bytes,
                       hipStream_t stream);
int nof_plan_autotune(nof_plan plan, const void* B, const double* C, const double* H,
                      const double* n, const double* cJ, const double* cK, double* E,
                      double* lambda, double* grad, void* ws, size_t ws_bytes,
                      hipStream_t stream);
int nof_plan_capture(nof_plan plan, const void* B, const double* C, const double* H,
                     const double* n, const double* cJ, const double* cK, double* E,
                     double* lambda, double* grad, void* ws, size_t ws_bytes,
                     hipStream_t stream);
int nof_plan_launch(nof_plan plan, hipStream_t stream);
int nof_plan_destroy(nof_plan plan);


/* ---------------------------------------------------------------------------
 * Learned warm start of the occupation update (not part of the paper's method:
 * its prediction is always refined by nof_occ_optimize).
 *
 * Network: 5 -> 128 -> 128 -> 1, tanh hidden units, output angle
 * theta = (pi/2) sigmoid(z) with n = cos^2 theta.  params is one FP32 vector of
 * nof_mlp_nparams() values: W1 [5][128], b1 [128], W2 [128][128], b2 [128],
 * w3 [128], b3 (row-major, inputs first: h1 = tanh(x W1 + b1)).
 *
 * nof_mlp_features: X [norb][5] FP32 = per-feature z-scores over the orbitals
 *   of (J_pp, K_pp, h_pp, mean_q J_pq, mean_q K_pq); h_pp = hdiag[p*hstride];
 *   ws: nof_mlp_features_ws(norb) bytes.
 * nof_mlp_targets: theta = arccos(sqrt(n)) (FP32) for n [count] (FP64, clamped
 *   to [0, 1]): the training target whose cos^2 is the occupation.
 * nof_mlp_forward: theta [rows] for X [rows][5].
 * nof_mlp_loss_grad: loss = mean_r (theta_r - target_r)^2 (device scalar, may
 *   be NULL) and its gradient grad [nparams]; partial sums per block of 64
 *   rows are reduced in a fixed order in FP64.  ws: nof_mlp_ws(rows) bytes.
 * nof_mlp_adam: in-place ADAM step on params with FP32 moments m, v (t >= 1).
 * nof_mlp_warm_gamma: variables gamma [ns][ng] (FP64) of the occupation map
 *   from predicted angles: n = cos^2 theta rescaled to sum to one in each
 *   subspace, every share raised to at least nfloor (0 <= nfloor < 1/(ng+1))
 *   and renormalised (with n_g raised to 1/2 for the trigonometric map), then
 *   the inverse map (softmax: gamma_i = ln(n_{p_i}/n_g)).  ng <= 64.  Bad
 *   member indices set info[2] = NOF_E_ARG (info may be NULL).
 * ------------------------------------------------------------------------- */
int nof_mlp_nparams(void);
size_t nof_mlp_ws(int rows);
size_t nof_mlp_features_ws(int norb);
int nof_mlp_features(int norb, const double* hdiag, int hstride, const double* J,
                     const double* K, float* X, void* ws, size_t ws_bytes, hipStream_t stream);
int nof_mlp_targets(int n, const double* occ, float* theta, hipStream_t stream);
int nof_mlp_forward(int rows, const float* X, const float* params, float* theta,
                    hipStream_t stream);
int nof_mlp_loss_grad(int rows, const float* X, const float* target, const float* params,
                      float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t stream);
int nof_mlp_adam(int nparams, float* params, const float* grad, float* m, float* v, int t,
                 float lr, float beta1, float beta2, float eps, hipStream_t stream);
int nof_mlp_warm_gamma(int norb, int ns, int ng, const int* members, int map,
                       const float* theta, double nfloor, double* gamma, int* info,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * The alternating NO + ON optimisation to convergence (Theory: the energy is
 * minimised separately over occupations and orbitals; Occupation Number
 * Optimization; Natural Orbital Optimization: lambda symmetric at the
 * minimum, g = 4(lambda - lambda^T), ADAM on the generator y, U = exp(y)).
 *
 * Outer iteration: the ON step at fixed orbitals (nof_occ_optimize on gamma
 * with h, J, K of the current C; skipped when on_maxit = 0, the occupations
 * then stay those of gamma), then a sweep of up to no_steps ADAM steps
 * C <- C exp(y) at fixed occupations.  A sweep ends once
 * max|lambda - lambda^T| <= tol_lambda (NTHRESHL's criterion); the run ends
 * when a sweep ended so and E changed by at most tol_energy since the
 * previous outer iteration (NTHRESHE's), or after max_outer iterations.  The
 * ADAM moments persist over the run (one step counter for the bias
 * correction).  After every sweep nof_orthonormalize checks C^T C = I and
 * repairs C when max|C^T C - I| > tol_orth.  The host reads E and
 * max|lambda - lambda^T| once per step and the check once per sweep.
 *
 * B, Bt, prec   as nof_mo_transform (NOF_P_F64, NOF_P_F32 or NOF_P_BF16X10;
 *               for X10, B in FP32 or as nof_split_B planes).
 * H             [nbf][nbf] FP64 AO one-electron matrix.
 * C             [nbf][norb] FP64, in: start orbitals, out: final orbitals.
 * members, map, func, ns, ng   as nof_occ_optimize (device).
 * gamma         [ns][ng] FP64, in/out.   n_out  [norb] FP64, may be NULL.
 * p             host parameters (typical: 100 outer, 30 steps, lr 0.01,
 *               0.9, 0.999, 1e-8, tol_lambda 1e-5, tol_energy 1e-9,
 *               on_maxit 2000, on_tol 1e-8, tol_orth 1e-10; tol_orth >= 0).
 * res           host result.  Errors: NOF_E_NULL, NOF_E_ARG, NOF_E_DIM,
 *               NOF_E_WORKSPACE, the status of a failing step (also in
 *               res->status), NOF_E_NOT_CONVERGED if E or the asymmetry
 *               stops being finite.  Not convergence within max_outer is
 *               not an error: res->converged = 0.
 * ws            at least nof_solve_ws(...) bytes.  Not capturable in a HIP
 *               graph (it synchronises the stream every step).
 * ------------------------------------------------------------------------- */
/* orbopt: 1 = each NO step is one step of nof_pseudo_fock_diag (iterative
 * diagonalization, IORBOPT = 1; its diagonal persists over the run, lambda_pp
 * at the first step) with off-diagonal bound maxoff; any other value = ADAM
 * rotation steps (IORBOPT = 2). */
typedef struct {
  int max_outer, no_steps;
  double lr, beta1, beta2, eps;
  double tol_lambda, tol_energy;
  int on_maxit;
  double on_tol;
  double tol_orth;
  int orbopt;
  double maxoff;
} nof_solve_params;

/* orth: the largest max|C^T C - I| that the checks after the sweeps found.
 * on_unconverged: ON steps (nof_occ_optimize calls) that stopped at on_maxit
 * without meeting their stopping test.  converged = 1 needs the run's
 * criteria and a converged ON step in the last outer iteration. */
typedef struct {
  double E, asym;
  int outer, no_steps, on_iters, converged, status;
  double orth;
  int on_unconverged;
} nof_solve_result;

size_t nof_solve_ws(int naux, int nbf, int norb, int ns, int ng, int Bt, int prec);
int nof_solve(int naux, int nbf, int norb, const void* B, int Bt, const double* H, double* C,
              int ns, int ng, const int* members, int map, int func, double* gamma,
              double* n_out, int prec, const nof_solve_params* p, nof_solve_result* res,
              void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched solve (NLOPs: Polarizabilities and Hyperpolarizabilities: the
 * finite-field instances share B and differ in H): the alternating NO + ON
 * optimisation of nof_solve, run for every instance of a plan at once.
 *
 * Per outer iteration: one batched iteration gives h_i, J_i, K_i of the
 * current orbitals; each instance still running takes its ON step
 * (nof_occ_optimize, or the occupations of gamma_i when on_maxit = 0) and its
 * coefficients; then NO steps until every instance's sweep has ended.  A NO
 * step of all instances is the batched iteration, max|lambda_i - lambda_i^T|
 * per instance, ADAM on the instances whose sweep runs and whose asymmetry is
 * above tol_lambda, U_i = exp(y_i) and C_i <- C_i U_i; the other instances get
 * y_i = 0 and keep C_i bit for bit.  With a non-null stream the NO step is
 * captured once into a HIP graph and each step is one hipGraphLaunch; the
 * host reads E_i and the asymmetries after every step.  Every instance
 * follows the same sequence of states as nof_solve would give it alone
 * (sweep and convergence rules, ADAM moments and step counter per instance).
 *
 * plan     from nof_plan_create (any of its precisions; B as for
 *          nof_plan_iteration).  Uses the plan's tuned configuration; the
 *          plan's own captured graph, if any, is left alone.
 * H        [ninst][nbf][nbf] FP64; C [ninst][nbf][norb] FP64 in/out.
 * members, map, func, ns, ng   as nof_occ_optimize, shared by all instances.
 * gamma    [ninst][ns][ng] FP64 in/out.  n_out [ninst][norb] or NULL.
 * p        host parameters as nof_solve (ADAM steps only: orbopt = 1 is
 *          NOF_E_ARG).  res [ninst] host results.
 * ws       nof_plan_solve_ws(plan, ns, ng) bytes (includes the plan's).
 * Returns NOF_E_NOT_CONVERGED when an instance's E or asymmetry stopped being
 * finite (that instance stops, res[i].status says so, the others run on),
 * the status of a failing step otherwise, else NOF_OK.  Synchronises stream.
 * ------------------------------------------------------------------------- */
size_t nof_plan_solve_ws(nof_plan plan, int ns, int ng);
int nof_plan_solve(nof_plan plan, const void* B, const double* H, double* C, int ns, int ng,
                   const int* members, int map, int func, double* gamma, double* n_out,
                   const nof_solve_params* p, nof_solve_result* res, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Finite-field NLOPs (NLOPs: Polarizabilities and Hyperpolarizabilities).
 *
 * nof_dipole: electronic dipole of a NOF state along one axis,
 *   mu = -2 sum_p n_p (C^T d C)_pp,
 * for a field entering as H(F) = H + F d (d: AO matrix of the coupling, minus
 * the dipole operator; at a converged state mu = -dE/dF).  C [nbf][norb],
 * n [norb], d [nbf][nbf] FP64 device; mu out, one FP64 device scalar.
 * ws: nof_dipole_ws() bytes.
 *
 * nof_nlop_romberg: alpha = dmu/dF, beta = d^2mu/dF^2, gamma = d^3mu/dF^3
 * at F = 0 from the dipoles on the dyadic ladder h_k = step 2^(k-1):
 *   alpha(h) = (mu(h) - mu(-h)) / 2h,  beta(h) = (mu(h) - 2mu(0) + mu(-h)) / h^2,
 *   gamma(h) = (mu(2h) - 2mu(h) + 2mu(-h) - mu(-2h)) / 2h^3,
 *   R(k,1) = D(h_k),  R(k,j) = R(k,j-1) + (R(k,j-1) - R(k+1,j-1)) / (4^(j-1) - 1);
 * the value is R(k,j+1) of the vertical pair (k,k+1) of column j with the
 * smallest |R(k+1,j) - R(k,j)| (its uncertainty); equal differences go to the
 * candidate of smallest magnitude.
 * mu0       device scalar mu(0).
 * mu_p, mu_m [npoint+1] device: mu(+h_k), mu(-h_k), k = 1..npoint+1.
 * table     out [3][npoint][npoint] (alpha, beta, gamma; NaN outside the
 *           triangle, row k = step index, column j = extrapolation order).
 * result    out [3][4]: value, uncertainty, k, j (0-based; npoint = 1: the
 *           first estimate, uncertainty NaN).
 * Errors: NOF_E_DIM (npoint outside 1..16), NOF_E_ARG (step <= 0), NOF_E_NULL.
 * ------------------------------------------------------------------------- */
size_t nof_dipole_ws(int nbf, int norb);
int nof_dipole(int nbf, int norb, const double* C, const double* n, const double* d, double* mu,
               void* ws, size_t ws_bytes, hipStream_t stream);
int nof_nlop_romberg(int npoint, double step, const double* mu0, const double* mu_p,
                     const double* mu_m, double* table, double* result, hipStream_t stream);
/* Isotropic polarizability and anisotropy (Raman convention, ISOALPHA) of the
 * diagonal components alpha[3] (xx, yy, zz; device): out[0] = mean,
 * out[1] = sqrt(((a_xx - a_yy)^2 + (a_yy - a_zz)^2 + (a_zz - a_xx)^2) / 2). */
int nof_nlop_isotropic(const double* alpha, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* NOF_H */
