// Shared device/host helpers of the HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "nof.h"

namespace nof {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Round a byte count up to a 256-byte boundary (workspace sub-buffers).
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Host-side status from the last launch.
inline int launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? NOF_OK : NOF_E_HIP;
}

inline size_t dtype_size(int t) {
  switch (t) {
    case NOF_F64: return 8;
    case NOF_F32: return 4;
    case NOF_BF16: return 2;
    case NOF_BF16X4: return 8;                 // four planes (padded rows)
    case NOF_I8X4: return 4;                   // four INT8 planes (and row exponents)
    default: return 0;
  }
}

// ---------------------------------------------------------------------------
// Internal launchers (defined in the .hip files, called by api.hip).
// ---------------------------------------------------------------------------

// Batched "TN" matrix product on the matrix cores:
//   Out_b[m][n] = sum_k X_b(k, m) * Y_b(k, n) * S(k, n)
// X_b(k,m) = X[b*sx + k*ldx + m]            (x_kmajor)
//          = X[b*sx + m*ldx + k]            (!x_kmajor)
// Y_b(k,n) = Y[b*sy + k*ldy + n];  S optional (FP64, shared by all b).
// sym:  only tiles with tile_m <= tile_n are computed; elements with m <= n
//       are written to Out[m][n] and Out[n][m]; Dg[b*sd + m] = Out[m][m].
// fold: batches [c*fold, (c+1)*fold) are accumulated into one result that is
//       written to Out + c*so (split reduction over the batch index).
enum class GemmRole : int { Small = 0, TransformStage1, TransformStage2, ExchangeFock };

struct GemmDesc {
  int M, N, K;
  long long Ktot;    // if > 0: batch b only has k < Ktot - b*K (split-K over batches)
  int batch;        // number of batches b
  int fold;         // 1 = independent batches; >1 = accumulate groups of batches
  const void* X; long long ldx, sx; bool x_kmajor;
  const void* Y; long long ldy, sy;
  const double* S; long long lds;
  void* Out; long long ldo, so;
  double* Dg; long long sd;
  bool sym;
  const int* pred; int pred_gt;   // if pred: run only when *pred > pred_gt (else write nothing);
  long long pred_so;               // with two-level batching, outer index o reads pred[o * pred_so]
  GemmRole role;                   // selects the kernel symbol (profiling attribution only)
  long long psx, psy;              // plane strides of pre-split bf16 operands (gemm_bf16)
  // Two-level batching (binner > 0): batch b = outer * binner + inner; operand
  // offsets inner * s? + outer * s?2; fold groups never cross an outer index,
  // and with fold > 1 partial results go to Out + group * so.
  int binner;
  long long sx2, sy2, so2, sd2, ss2;
  int tile;                        // workgroup tile edge of gemm_tn: 128 (default) or 64
  // Exchange-type role with S only: if W, the right operand becomes
  // Y_b(k,n) S(k,n) - [k == n] W[outer*sw2 + b*ldw + n], so that the product
  // is the exchange-type term minus the Coulomb-type term (F2 - F1).
  const double* W; long long ldw, sw2;
};

// Element types: 0 = f64, 1 = f32.  prec: NOF_P_F64 or NOF_P_F32.
// X,Y element types given separately so that an FP64 master copy (C) can be
// consumed by an FP32 contraction.  Out type: f64 or f32.
int gemm_tn(const GemmDesc& d, int x_t, int y_t, int out_t, int prec, hipStream_t st);

// Split-precision BF16 form of the same contract (gemm_bf16.hip); prec is one
// of NOF_P_BF16X1/X3/X6/X10; x_t may be NOF_BF16 for the first transform stage.
int gemm_bf16(const GemmDesc& d, int x_t, int y_t, int out_t, int prec, hipStream_t st);
// Split a k-major FP64 matrix into np bf16 planes [np][ncol][ldk] (gemm_bf16.hip).
// Fixed-point (x10) transform stage on the matrix cores (gemm_fx.hip):
//   Out_b[m][n] = sum_k X_b(k, m) Y_b(k, n)   (FP32 out, FP64 diagonal Dg if sym)
// X: planes [4][..] at X + q*psx + b*sx + m*ldx + k, or FP32 at X + b*sx + k*ldx + m
//    with row grid exponents ex[b*sex + m];  Y likewise (n for m, ey/sey).
struct FxDesc {
  int M, N, K, batch;
  const void* X; long long ldx, sx, psx; const int* ex; long long sex;
  const void* Y; long long ldy, sy, psy; const int* ey; long long sey;
  float* Out; long long ldo, so;
  double* Dg; long long sd;
  bool sym;
  int role;                        // 1 = transform stage 1, 2 = stage 2 (kernel symbol)
  bool x_rows;                     // FP32 X symmetric per batch: may be read m-major (rows)
  unsigned* cmax; long long scm;   // optional: per row tile t the FP32 bits of max_m |Out_b[m][n]|
                                   // over the tile's rows -> cmax[b*scm + t*N + n] (not sym)
  // Two-level batching (binner > 0, not with cmax): batch b = outer * binner +
  // inner; X, Y, ey, Out, Dg at inner * s? + outer * s?2
  int binner = 0;
  long long sx2 = 0, sy2 = 0, sey2 = 0, so2 = 0, sd2 = 0;
  int tile = 128;                  // workgroup tile edge: 128, or 64 with pre-split X
  // Slabs folded into rows (X as planes, batch 1, not sym): M = nslab * mslab
  // rows, slab b = rows b*mslab.., mslab >= tile.  cmax then keeps per row
  // tile t the maxima over the rows of its first slab at cmax[t*N + n] and,
  // for a tile that reaches into slab b + 1, over those rows at
  // cmax[scm + (b+1)*N + n] (scm = row tiles * N); see cmax_words.
  int mslab = 0;
};
int gemm_fx(const FxDesc& d, bool x_planes, bool y_planes, hipStream_t st);
// Column grid exponents e[b*N + n] from the row-tile maxima above.
// mslab > 0: cmax of a folded product over `batch` slabs of mslab rows,
// `tiles` its row tiles at edge ts.
int fx_cmax_exps(const unsigned* cmax, int batch, int tiles, int N, int* e, hipStream_t st, int mslab = 0,
                 int ts = 128);
// Row tiles of n rows at tile edge ts (the cmax layout).
inline int fx_tiles(int n, int ts = 128) { return (n + ts - 1) / ts; }
// cmax words of a stage-1 product over nslab slabs of mslab rows and N
// columns at tile edge ts: per slab (folded = false) or with the slabs'
// rows folded into one M (folded = true, mslab >= ts).
inline long long cmax_words(long long nslab, int mslab, long long N, int ts, bool folded) {
  return folded ? ((nslab * mslab + ts - 1) / ts + nslab) * N : nslab * fx_tiles(mslab, ts) * N;
}
// Largest column maximum of slab b (column n) from a folded cmax: the row
// tiles that start inside the slab, and the tile that starts in slab b - 1
// and reaches into it (when the slab does not start on a tile edge).
__device__ inline unsigned slab_cmax(const unsigned* cmax, long long b, int mslab, int ts, long long tiles,
                                     int N, int n) {
  const long long r0 = b * mslab;
  unsigned m = 0;
  for (long long t = (r0 + ts - 1) / ts; t * ts < r0 + mslab; ++t) m = max(m, cmax[t * N + n]);
  if (r0 % ts) m = max(m, cmax[(tiles + b) * N + n]);
  return m;
}
// INT8 fixed-point transform stage (gemm_i8.hip, NOF_P_I8X10):
//   Out_b[m][n] = sum_k X_b(k, m) Y_b(k, n)   (FP32 out, FP64 diagonal Dg if sym)
// X: INT8 planes at X + q*psx + b*sx + m*ldx + k (ldx a multiple of 64, zero
// for k >= K) with grid exponents ex[b*sex + m]; Y likewise (n, ey, sey).
// cmax as in FxDesc.
constexpr int I8_MAX_K = 65536;          // int32 sums of the pieces stay exact below this depth
struct I8Desc {
  int M, N, K, batch;
  const unsigned char* X; long long ldx, sx, psx; const int* ex; long long sex;
  const unsigned char* Y; long long ldy, sy, psy; const int* ey; long long sey;
  float* Out; long long ldo, so;
  double* Dg; long long sd;
  bool sym;
  int role;                        // 1 = transform stage 1, 2 = stage 2 (kernel symbol)
  unsigned* cmax; long long scm;
  // Two-level batching (binner > 0, not with cmax): batch b = outer * binner +
  // inner; X, ex, Y, ey, Out, Dg at inner * s? + outer * s?2
  int binner;
  long long sx2, sex2, sy2, sey2, so2, sd2;
  double* Out64;                   // if set (no cmax, no Dg): FP64 results here instead of Out
                                   // (sym: both triangles)
  int mslab;                       // slabs folded into rows, as in FxDesc (tile edge 128)
};
int gemm_i8(const I8Desc& d, hipStream_t st);
// Exchange-type Fock partials of the INT8 form (gemm_i8.hip):
//   Out[i][g][r][s] = sum_{P in group g} sum_q b_i^P[q][r] St_i[s][q] b_i^P[q][s]
// as one INT8 product per group of `fold` slabs (grids per group and row,
// exact int32 sums over the group, FP64 out).  b FP32 [ninst][naux][norb][norb]
// (instance stride sb), St FP32 [ninst][norb][norb]; ws of i8_exchange_ws bytes.
int i8_exchange_fold(int naux, int norb);
size_t i8_exchange_ws(int ninst, int naux, int norb);
int i8_exchange(int ninst, int naux, int norb, const float* b, long long sb, const float* St, double* Out,
                void* ws, hipStream_t st);
inline long long i8_ldk(int K) { return ((long long)K + 63) / 64 * 64; }
// Bytes of the four INT8 planes of rows x K (the grid exponents follow at this offset).
inline size_t i8_planes_bytes(long long rows, int K) { return align256((size_t)4 * rows * i8_ldk(K)); }
// INT8 planes [4][nrow][ldk] and grid exponents e[nrow] of the rows of
// A[nrow][K] (FP64/FP32); of the columns of an FP64 k-major A[k][col]
// ([4][ncol][ldk], e[ncol]); grid exponents of T_b's columns from the stage-1
// column maxima; planes [4][batch][N][ldk] of the columns of the k-major FP32
// T_b[K][N] on those grids.
int i8_split_rows(const void* A, int At, long long nrow, int K, int ldk, void* planes, int* e,
                  hipStream_t st);
int i8_split_cols(const double* A, int K, int ncol, int lda, int ldk, void* planes, int* e,
                  hipStream_t st);
int i8_cmax_exps(const unsigned* cmax, int batch, int tiles, int N, int* e, hipStream_t st, int mslab = 0);
int i8_split_T(const float* T, int batch, int K, int N, long long sT, int ldk, const int* e, void* planes,
               hipStream_t st, long long ldt = 0);
// Grids of the per-q products of the INT8 exchange-type term: e[q*norb + r]
// from max_P |b^P[q][r]| (FP32 b [naux][norb][norb]).
int i8_slab_grids(const float* b, int naux, int norb, int* e, hipStream_t st);

// Exchange-type Fock partials of the split forms (gemm_fx.hip):
//   Out[g][r][s] = sum_{P in [g*fold, (g+1)*fold)} sum_q b^P[q][r] S[q][s] b^P[q][s]
// b FP32 [naux][norb][norb] symmetric slabs; S FP64 [norb][norb]; St a
// norb*norb FP32 scratch (S transposed); Out FP64 [groups][norb][norb].
// ninst > 1: instance i reads b + i*sb, S + i*norb^2 and writes Out + i*so;
// St then holds ninst transposed copies (norb^2 apart).
struct ExDesc {
  int naux, norb, fold;
  const float* b;
  const float* St;
  double* Out;
  int ninst = 1;
  long long sb = 0, so = 0;
  int tile = 128;                  // workgroup tile edge, 128 or 64
};
int exchange_fock_fx(const ExDesc& d, const double* S, float* St, hipStream_t st);
// St_i[s][q] = (float)S_i[q][s] for ninst matrices n^2 apart.
int fx_transpose(const double* S, int n, int ninst, float* St, hipStream_t st);
// Grid exponents (2^E above the largest |value|) of rows of A[nrow][K] (FP64/FP32)
// and of the columns of A_b[K][N] (FP32, batch stride sa) -> e[b*N + n].
int fx_row_exps(const void* A, int At, long long nrow, int K, int* e, hipStream_t st);
int fx_col_exps(const float* A, int batch, int K, int N, long long sa, int* e, hipStream_t st);
// Four fixed-point planes: of the columns of an FP64 k-major A[k][col] -> [4][ncol][ldk],
// and of the rows of A[nrow][K] (FP64/FP32) -> [4][nrow][ldk]; zero for k >= K.
int fx_split_cols(const double* A, int K, int ncol, int lda, int ldk, void* out, hipStream_t st);
int fx_split_rows(const void* A, int At, long long nrow, int K, int ldk, void* out, hipStream_t st);
int presplit_bf16(const double* A, int K, int ncol, int lda, int ldk, int np, void* out,
                  hipStream_t st);
inline int bf16_pieces(int prec) {
  return prec == NOF_P_BF16X1 ? 1 : prec == NOF_P_BF16X3 ? 2 : prec == NOF_P_BF16X10 ? 4 : 3;
}
inline long long presplit_ldk(int K) { return ((long long)K + 31) / 32 * 32; }

inline bool is_bf16_prec(int prec) {
  return prec == NOF_P_BF16X1 || prec == NOF_P_BF16X3 || prec == NOF_P_BF16X6 ||
         prec == NOF_P_BF16X10;
}
inline int gemm_any(const GemmDesc& d, int x_t, int y_t, int out_t, int prec, hipStream_t st) {
  return is_bf16_prec(prec) ? gemm_bf16(d, x_t, y_t, out_t, prec, st)
                            : gemm_tn(d, x_t, y_t, out_t, prec, st);
}

// Pass over the upper triangle of b (HBM bound), written as nparts partial
// planes whose in-order sum is
//   K[r][s] = sum_P b_rs^2                                     (r <= s)
//   F1[r][s] = sum_P b_rs W[P][s],  F1[s][r] = sum_P b_rs W[P][r]
// Either output may be NULL.  nparts must equal kf1_parts(naux, norb, ninst,
// bt); every element of every plane that the sum reads is written (no
// clearing).
int kf1_pass(int naux, int norb, const void* b, int bt, const double* W,
             double* Kpart, double* F1part, int nparts, hipStream_t st, int ninst = 1,
             long long bstride = 0, long long wstride = 0, long long pstride = 0);
int kf1_parts(int naux, int norb, int ninst, int bt);

// out[i] = sum_c part[c*stride + i] in fixed order; if sym_upper, element
// (r,s) is read from (min,max) and written to both (r,s) and (s,r).
int reduce_parts(const double* part, int nparts, long long stride, int norb,
                 bool sym_upper, double* out, hipStream_t st, int ninst = 1,
                 long long pinst = 0, long long oinst = 0);

// F[r][s] = start + sum_{q < qn} cK[q][s] G[q][r][s] in q order (G: qn FP64
// norb x norb matrices; cK: the qn rows of the coefficients that go with
// them); start = 0 (mode 0), F (mode 1) or -F1 (mode 2).  ninst instances:
// G, cK, F1 / F at the given strides.
int exchange_accum(const double* G, int qn, int norb, const double* cK, const double* F1, int mode,
                   double* F, hipStream_t st, int ninst = 1, long long gstride = 0, long long cstride = 0,
                   long long fstride = 0);
// q values per chunk of the per-q products G^q of ninst instances within
// 4 GiB (fewer, larger launches: at Norb = 1000 two launches of 536 and 464
// values of q ran 3 % faster than eight of 134 within 1 GiB).
inline int exchange_sym_chunk(int norb, int ninst = 1) {
  const long long per = (long long)norb * norb * (long long)sizeof(double) * ninst;
  long long c = (4LL << 30) / per;
  if (c < 1) c = 1;
  if (c > norb) c = norb;
  return (int)c;
}

// y -= x (n elements; ninst instances at the given strides).
int subtract(long long n, const double* x, double* y, hipStream_t st, int ninst = 1,
             long long xstride = 0, long long ystride = 0);

// Instance-batched forms (grid dimension over instances with the given strides).
int lambda_grad(int norb, const double* n, const double* h, const double* F1,
                const double* F2, double* lam, double* grad, hipStream_t st, int ninst = 1,
                long long nstride = 0, long long mstride = 0, long long fstride = 0);

// E of ninst instances; part: energy_ws(ninst) bytes of partial sums.
size_t energy_ws(int ninst);
int energy(int norb, const double* n, const double* h, const double* J,
           const double* K, const double* cJ, const double* cK, double* E, double* part,
           hipStream_t st, int ninst = 1, long long nstride = 0, long long mstride = 0,
           long long jstride = 0);

// FP64 orbital-rotation helpers (rotation.hip).
size_t expm_ws(int norb, int ninst = 1);
size_t rotate_ws(int nbf, int norb, int ninst = 1);
// ninst instances at once: C, Cout stride nbf*norb, U and y stride norb^2;
// ws of rotate_ws / expm_ws(.., ninst) bytes.
int rotate_orbitals(int nbf, int norb, const double* C, const double* U, double* Cout, void* ws,
                    hipStream_t st, int ninst = 1);
int expm_antisym(int norb, const double* y, double* U, void* ws, hipStream_t st, int ninst = 1);
// Orthonormality check and repair of C [nbf][norb] (S [nbf][nbf] or NULL):
// err = max|C^T S C - I| (device, may be NULL); C <- C (I - E/2) when err > tol.
size_t orth_ws(int nbf, int norb);
int orthonormalize(int nbf, int norb, double* C, const double* S, double tol, double* err, void* ws,
                   hipStream_t st);
int adam_step(int norb, const double* g, double* m, double* v, int t, double lr, double beta1,
              double beta2, double eps, double* y, hipStream_t st);

// Occupation update (occupations.hip).
size_t occ_ws(int norb, int ns, int ng);
int occ_energy_grad(int norb, int ns, int ng, const int* members, int map, int func,
                    const double* gamma, const double* hdiag, int hstride, const double* J,
                    const double* K, double* n, double* E, double* dEdgamma, int* info, void* ws,
                    hipStream_t st);
int occ_optimize(int norb, int ns, int ng, const int* members, int map, int func,
                 const double* hdiag, int hstride, const double* J, const double* K,
                 double* gamma, double* n, double* E, int* info, int maxit, double tol, void* ws,
                 hipStream_t st);
int functional_coeffs(int norb, int ns, int ng, const int* members, int func, const double* n,
                      double* cJ, double* cK, void* ws, int* bad, hipStream_t st);
// ON steps of ninst independent problems in one launch (one workgroup each):
// instance i reads hdiag + i*hinst, J, K + i*jkinst, updates gamma + i*ns*ng,
// writes n + i*norb, E[i], info[3i..3i+2] and uses workspace
// ws + i*occ_ws_stride(); skipped when active[i] == 0 (active may be NULL).
// maxit > 0: L-BFGS as occ_optimize; maxit == 0: evaluation only.
size_t occ_ws_stride(int norb, int ns, int ng);
int occ_batched(int ninst, const int* active, int norb, int ns, int ng, const int* members, int map,
                int func, const double* hdiag, int hstride, long long hinst, const double* J,
                const double* K, long long jkinst, double* gamma, double* n, double* E, int* info,
                int maxit, double tol, void* ws, hipStream_t st);

// Learned warm start (mlp.hip).
int mlp_nparams();
int mlp_targets(int n, const double* occ, float* theta, hipStream_t st);
size_t mlp_ws(int rows);
int mlp_forward(int rows, const float* X, const float* P, float* theta, hipStream_t st);
int mlp_loss_grad(int rows, const float* X, const float* target, const float* P, float* grad,
                  float* loss, void* ws, hipStream_t st);
int mlp_adam(int n, float* p, const float* g, float* m, float* v, int t, float lr, float b1,
             float b2, float eps, hipStream_t st);
int mlp_features(int norb, const double* hdiag, int hstride, const double* J, const double* K,
                 float* X, void* ws, hipStream_t st);
int mlp_warm_gamma(int norb, int ns, int ng, const int* members, int map, const float* theta,
                   double nfloor, double* gamma, int* info, hipStream_t st);

int coeffs_from_cumulant(int norb, const double* n, const double* Delta,
                         const double* Pi, double* cJ, double* cK, hipStream_t st);

}  // namespace nof
