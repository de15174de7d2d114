// Batched form: many instances that share the three-index tensor B but carry
// their own orbitals C_i, one-electron matrix H_i, occupations and
// coefficients (e.g. the finite-field instances of the nonlinear-optics
// workflow: H_i = H + F_i d, one field per instance).
//
// One iteration for all instances:
//   1. the C_i are packed side by side, C_all[nu][i*norb + q], so the first
//      transform stage reads B once for every instance: T_all = B^P C_all;
//   2. b_i^P = C_i^T T_i^P, D_i (one launch over (instance, P));
//   3. h_i = C_i^T H_i C_i, J_i = D_i^T D_i, W_i = D_i cJ_i (instance-batched);
//   4. one pass over every b_i for K_i and the Coulomb-type term;
//   5. the exchange-type term per instance (split over P), lambda_i, g_i, E_i.
// Every step is an instance-batched launch on the caller's stream, so the
// iteration can be captured once into a HIP graph and replayed with a single
// hipGraphLaunch.  The workgroup tile of each matrix product (128 or 64) and
// the P-split of the exchange term are chosen by timing the candidates
// (nof_plan_autotune).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "common.h"

namespace nof {
// Regions of a plan's workspace (byte offsets in nof_plan_s::off).
enum PlanRegion : int {
  O_CALL = 0, O_T, O_B, O_D, O_TH, O_H, O_J, O_K, O_W, O_KP, O_F1P, O_F2P, O_F1, O_F2, O_EP,
  O_CPL, O_CMX, O_EY, O_ST,          // the fixed-point forms only
  O_TPL,                             // the INT8 form only: T as planes
  O_N
};
}  // namespace nof

struct nof_plan_s {
  int ninst, naux, nbf, norb, prec, bt;
  int tile_s1, tile_s2, tile_f2, f2gpi;    // tuned choices
  int kchunks;
  size_t off[nof::O_N];                    // one offset per region
  size_t bytes[nof::O_N];                  // and its size
  size_t total;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
};

namespace nof {
namespace {

// The fixed-point forms (BF16 or INT8 pieces) share b in FP32, the x10
// exchange-type product and the Coulomb-type term from the pass.
bool fixed_point_plan(const nof_plan_s* p) { return p->prec == NOF_P_BF16X10 || p->prec == NOF_P_I8X10; }
// Plans whose Coulomb-type term comes from the pass over b (with K): the
// fixed-point ones and FP64 (exchange-type term through the per-q products).
bool f1_pass_plan(const nof_plan_s* p) { return fixed_point_plan(p) || p->prec == NOF_P_F64; }
// Stage 1 of the fixed-point plans takes the rows of all slabs as one M when
// a slab holds at least one tile of rows: no slab is padded to whole tiles.
bool fold_stage1(const nof_plan_s* p, int tile) {
  return p->nbf >= tile && (long long)p->naux * p->nbf + p->nbf <= 0x7fffffffLL;
}
long long stage1_cmax_words(const nof_plan_s* p, int tile) {
  return cmax_words(p->naux, p->nbf, (long long)p->ninst * p->norb, tile, fold_stage1(p, tile));
}

void plan_layout(nof_plan_s* p) {
  const size_t ni = p->ninst, na = p->naux, nb = p->nbf, no = p->norb;
  const size_t es = dtype_size(p->bt);
  const size_t n2 = no * no * 8;
  const int f2groups = p->ninst * p->f2gpi;
  size_t sz[O_N];
  sz[O_CALL] = nb * ni * no * 8;
  sz[O_T] = na * nb * ni * no * es;
  sz[O_B] = ni * na * no * no * es;
  sz[O_D] = ni * na * no * 8;
  sz[O_TH] = ni * nb * no * 8;
  sz[O_H] = ni * n2;
  sz[O_J] = ni * n2;
  sz[O_K] = ni * n2;
  sz[O_W] = ni * na * no * 8;
  sz[O_KP] = ni * p->kchunks * n2;
  // F32: the Coulomb-type term is folded into the exchange-type product
  // (O_F2 holds F2 - F1), so its partials and sum take no space; the FP64 and
  // fixed-point exchange-type terms do not take it (F1 from the pass with K).
  // FP64: O_F2P holds a chunk of the per-q products G^q of every instance.
  const bool fx1 = f1_pass_plan(p);
  sz[O_F1P] = fx1 ? ni * p->kchunks * n2 : 0;
  sz[O_F2P] = p->prec == NOF_P_F64 ? ni * (size_t)exchange_sym_chunk(p->norb, p->ninst) * n2
                                   : (size_t)f2groups * n2;
  sz[O_F1] = fx1 ? ni * n2 : 0;
  sz[O_F2] = ni * n2;
  sz[O_EP] = energy_ws((int)ni);
  // fixed-point forms: planes of the packed C (INT8: and their exponents),
  // column maxima of T per row tile, the grid exponents of T's columns,
  // every instance's cK transposed in FP32; INT8: T as planes
  const bool fx = fixed_point_plan(p);
  const bool i8 = p->prec == NOF_P_I8X10;
  const size_t ldk = (size_t)presplit_ldk(p->nbf), ldc = ni * no;
  sz[O_CPL] = !fx ? 0 : i8 ? i8_planes_bytes((long long)ldc, p->nbf) + ldc * 4 : 4 * ldc * ldk * 2;
  sz[O_CMX] = fx ? (size_t)std::max(stage1_cmax_words(p, 128),
                                     p->prec == NOF_P_BF16X10 ? stage1_cmax_words(p, 64) : 0LL) * 4
               : 0;
  sz[O_EY] = fx ? na * ldc * 4 : 0;
  sz[O_ST] = fx ? ni * no * no * 4 : 0;
  sz[O_TPL] = i8 ? i8_planes_bytes((long long)na * ldc, p->nbf) : 0;
  size_t o = 0;
  for (int i = 0; i < O_N; ++i) {
    p->off[i] = o;
    p->bytes[i] = sz[i];
    o = align256(o + sz[i]);
  }
  p->total = o;
}

__global__ void k_pack_C(int ninst, int nbf, int norb, const double* __restrict__ C,
                         double* __restrict__ Call) {
  const long long n = (long long)ninst * nbf * norb;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / ((long long)nbf * norb);
    const long long r = e - i * nbf * norb;
    const long long nu = r / norb, q = r - nu * norb;
    Call[nu * ninst * norb + i * norb + q] = C[e];
  }
}

struct Args {
  const void* B;
  const double *C, *H, *n, *cJ, *cK;
  double *E, *lam, *grad;
  char* ws;
};

// Stage kernels of one iteration.  Each returns a status.
int run_stage1(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long ldc = (long long)p->ninst * p->norb;
  if (p->prec == NOF_P_I8X10) {
    // B as INT8 planes with row exponents; the packed C split once into
    // INT8 planes of its ninst*norb columns; T's column maxima from the
    // epilogue give its grids, then T is split into planes of its columns
    const long long ldk = i8_ldk(p->nbf);
    unsigned char* cpl = (unsigned char*)(a.ws + p->off[O_CPL]);
    int* ce = (int*)(cpl + i8_planes_bytes(ldc, p->nbf));
    int rc = i8_split_cols((const double*)(a.ws + p->off[O_CALL]), p->nbf, (int)ldc, (int)ldc, (int)ldk,
                           cpl, ce, st);
    if (rc != NOF_OK) return rc;
    const unsigned char* Bp = (const unsigned char*)a.B;
    const bool fold = fold_stage1(p, 128);
    I8Desc f{};
    f.M = fold ? p->naux * p->nbf : p->nbf; f.N = (int)ldc; f.K = p->nbf; f.batch = fold ? 1 : p->naux;
    f.X = Bp; f.ldx = ldk; f.sx = fold ? 0 : (long long)p->nbf * ldk; f.psx = (long long)p->naux * p->nbf * ldk;
    f.ex = (const int*)(Bp + i8_planes_bytes((long long)p->naux * p->nbf, p->nbf)); f.sex = fold ? 0 : p->nbf;
    f.Y = cpl; f.ldy = ldk; f.sy = 0; f.psy = ldc * ldk; f.ey = ce; f.sey = 0;
    f.Out = (float*)(a.ws + p->off[O_T]); f.ldo = ldc; f.so = fold ? 0 : (long long)p->nbf * ldc;
    f.sym = false; f.role = 1; f.mslab = fold ? p->nbf : 0;
    const int rt = fx_tiles(f.M, 128);
    f.cmax = (unsigned*)(a.ws + p->off[O_CMX]); f.scm = (long long)rt * ldc;
    if ((rc = gemm_i8(f, st)) != NOF_OK) return rc;
    int* te = (int*)(a.ws + p->off[O_EY]);
    if ((rc = i8_cmax_exps(f.cmax, p->naux, rt, (int)ldc, te, st, f.mslab)) != NOF_OK) return rc;
    return i8_split_T(f.Out, p->naux, p->nbf, (int)ldc, (long long)p->nbf * ldc, (int)ldk, te,
                      a.ws + p->off[O_TPL], st);
  }
  if (p->prec == NOF_P_BF16X10) {
    // B as fixed-point planes [4][naux][nbf][ldk]; the packed C split once
    // into planes of its ninst*norb columns; the epilogue's column maxima of
    // T give stage 2 its grids
    const long long ldk = presplit_ldk(p->nbf);
    void* cpl = a.ws + p->off[O_CPL];
    int rc = fx_split_cols((const double*)(a.ws + p->off[O_CALL]), p->nbf, (int)ldc, (int)ldc, (int)ldk,
                           cpl, st);
    if (rc != NOF_OK) return rc;
    const bool fold = fold_stage1(p, p->tile_s1);
    FxDesc f{};
    f.M = fold ? p->naux * p->nbf : p->nbf; f.N = (int)ldc; f.K = p->nbf; f.batch = fold ? 1 : p->naux;
    f.X = a.B; f.ldx = ldk; f.sx = fold ? 0 : (long long)p->nbf * ldk; f.psx = (long long)p->naux * p->nbf * ldk;
    f.Y = cpl; f.ldy = ldk; f.sy = 0; f.psy = ldc * ldk;
    f.Out = (float*)(a.ws + p->off[O_T]); f.ldo = ldc; f.so = fold ? 0 : (long long)p->nbf * ldc;
    f.sym = false; f.role = 1; f.tile = p->tile_s1; f.mslab = fold ? p->nbf : 0;
    const int rt = fx_tiles(f.M, p->tile_s1);
    f.cmax = (unsigned*)(a.ws + p->off[O_CMX]); f.scm = (long long)rt * ldc;
    if ((rc = gemm_fx(f, true, true, st)) != NOF_OK) return rc;
    return fx_cmax_exps(f.cmax, p->naux, rt, (int)ldc, (int*)(a.ws + p->off[O_EY]), st, f.mslab, p->tile_s1);
  }
  GemmDesc g{};
  g.M = p->nbf; g.N = p->ninst * p->norb; g.K = p->nbf;
  g.batch = p->naux; g.fold = 1;
  g.X = a.B; g.ldx = p->nbf; g.sx = (long long)p->nbf * p->nbf; g.x_kmajor = true;
  g.Y = a.ws + p->off[O_CALL]; g.ldy = ldc; g.sy = 0;
  g.Out = a.ws + p->off[O_T]; g.ldo = ldc; g.so = (long long)p->nbf * ldc;
  g.role = GemmRole::TransformStage1;
  g.tile = p->tile_s1;
  return gemm_tn(g, p->bt, NOF_F64, p->bt, p->prec, st);
}

int run_stage2(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long ldc = (long long)p->ninst * p->norb;
  const long long n2 = (long long)p->norb * p->norb;
  if (p->prec == NOF_P_I8X10) {
    // instance i (outer index): its C planes are rows i*norb.. of the packed
    // planes, its T^P planes rows P*ldc + i*norb.., with their exponents
    const long long ldk = i8_ldk(p->nbf);
    const unsigned char* cpl = (const unsigned char*)(a.ws + p->off[O_CPL]);
    I8Desc f{};
    f.M = p->norb; f.N = p->norb; f.K = p->nbf;
    f.batch = p->ninst * p->naux; f.binner = p->naux;
    f.X = cpl; f.ldx = ldk; f.sx = 0; f.sx2 = (long long)p->norb * ldk; f.psx = ldc * ldk;
    f.ex = (const int*)(cpl + i8_planes_bytes(ldc, p->nbf)); f.sex = 0; f.sex2 = p->norb;
    f.Y = (const unsigned char*)(a.ws + p->off[O_TPL]); f.ldy = ldk; f.sy = ldc * ldk;
    f.sy2 = (long long)p->norb * ldk; f.psy = (long long)p->naux * ldc * ldk;
    f.ey = (const int*)(a.ws + p->off[O_EY]); f.sey = ldc; f.sey2 = p->norb;
    f.Out = (float*)(a.ws + p->off[O_B]); f.ldo = p->norb; f.so = n2; f.so2 = (long long)p->naux * n2;
    f.Dg = (double*)(a.ws + p->off[O_D]); f.sd = p->norb; f.sd2 = (long long)p->naux * p->norb;
    f.sym = true; f.role = 2;
    return gemm_i8(f, st);
  }
  if (p->prec == NOF_P_BF16X10) {
    // instance i (outer index): its C planes are columns i*norb.. of the
    // packed planes, its T^P columns i*norb.. of T, with their grid exponents
    const long long ldk = presplit_ldk(p->nbf);
    FxDesc f{};
    f.M = p->norb; f.N = p->norb; f.K = p->nbf;
    f.batch = p->ninst * p->naux; f.binner = p->naux;
    f.X = a.ws + p->off[O_CPL]; f.ldx = ldk; f.sx = 0; f.sx2 = (long long)p->norb * ldk; f.psx = ldc * ldk;
    f.Y = a.ws + p->off[O_T]; f.ldy = ldc; f.sy = (long long)p->nbf * ldc; f.sy2 = p->norb;
    f.ey = (const int*)(a.ws + p->off[O_EY]); f.sey = ldc; f.sey2 = p->norb;
    f.Out = (float*)(a.ws + p->off[O_B]); f.ldo = p->norb; f.so = n2; f.so2 = (long long)p->naux * n2;
    f.Dg = (double*)(a.ws + p->off[O_D]); f.sd = p->norb; f.sd2 = (long long)p->naux * p->norb;
    f.sym = true; f.role = 2; f.tile = p->tile_s2;
    return gemm_fx(f, true, false, st);
  }
  GemmDesc g{};
  g.M = p->norb; g.N = p->norb; g.K = p->nbf;
  g.batch = p->ninst * p->naux; g.fold = 1; g.binner = p->naux;
  g.X = a.C; g.ldx = p->norb; g.sx = 0; g.sx2 = (long long)p->nbf * p->norb; g.x_kmajor = true;
  g.Y = a.ws + p->off[O_T]; g.ldy = ldc; g.sy = (long long)p->nbf * ldc; g.sy2 = p->norb;
  g.Out = a.ws + p->off[O_B]; g.ldo = p->norb; g.so = n2; g.so2 = (long long)p->naux * n2;
  g.Dg = (double*)(a.ws + p->off[O_D]); g.sd = p->norb; g.sd2 = (long long)p->naux * p->norb;
  g.sym = true;
  g.role = GemmRole::TransformStage2;
  g.tile = p->tile_s2;
  return gemm_tn(g, NOF_F64, p->bt, p->bt, p->prec, st);
}

int run_small(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long n2 = (long long)p->norb * p->norb;
  double* Th = (double*)(a.ws + p->off[O_TH]);
  double* h = (double*)(a.ws + p->off[O_H]);
  double* D = (double*)(a.ws + p->off[O_D]);
  double* J = (double*)(a.ws + p->off[O_J]);
  double* W = (double*)(a.ws + p->off[O_W]);
  // h_i = C_i^T H_i C_i
  GemmDesc g1{};
  g1.M = p->nbf; g1.N = p->norb; g1.K = p->nbf; g1.batch = p->ninst; g1.fold = 1;
  g1.X = a.H; g1.ldx = p->nbf; g1.sx = (long long)p->nbf * p->nbf; g1.x_kmajor = true;
  g1.Y = a.C; g1.ldy = p->norb; g1.sy = (long long)p->nbf * p->norb;
  g1.Out = Th; g1.ldo = p->norb; g1.so = (long long)p->nbf * p->norb;
  int rc = gemm_tn(g1, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
  if (rc != NOF_OK) return rc;
  GemmDesc g2{};
  g2.M = p->norb; g2.N = p->norb; g2.K = p->nbf; g2.batch = p->ninst; g2.fold = 1;
  g2.X = a.C; g2.ldx = p->norb; g2.sx = (long long)p->nbf * p->norb; g2.x_kmajor = true;
  g2.Y = Th; g2.ldy = p->norb; g2.sy = (long long)p->nbf * p->norb;
  g2.Out = h; g2.ldo = p->norb; g2.so = n2; g2.sym = true;
  rc = gemm_tn(g2, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
  if (rc != NOF_OK) return rc;
  // J_i = D_i^T D_i
  GemmDesc gj{};
  gj.M = p->norb; gj.N = p->norb; gj.K = p->naux; gj.batch = p->ninst; gj.fold = 1;
  gj.X = D; gj.ldx = p->norb; gj.sx = (long long)p->naux * p->norb; gj.x_kmajor = true;
  gj.Y = D; gj.ldy = p->norb; gj.sy = (long long)p->naux * p->norb;
  gj.Out = J; gj.ldo = p->norb; gj.so = n2; gj.sym = true;
  rc = gemm_tn(gj, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
  if (rc != NOF_OK) return rc;
  // W_i = D_i cJ_i
  GemmDesc gw{};
  gw.M = p->naux; gw.N = p->norb; gw.K = p->norb; gw.batch = p->ninst; gw.fold = 1;
  gw.X = D; gw.ldx = p->norb; gw.sx = (long long)p->naux * p->norb; gw.x_kmajor = false;
  gw.Y = a.cJ; gw.ldy = p->norb; gw.sy = n2;
  gw.Out = W; gw.ldo = p->norb; gw.so = (long long)p->naux * p->norb;
  return gemm_tn(gw, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
}

// K of every instance in one pass over the upper halves of the b_i; in the
// x10 form also the Coulomb-type term F1 (same pass).
int run_pass(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long n2 = (long long)p->norb * p->norb;
  const bool fx = f1_pass_plan(p);
  double* kp = (double*)(a.ws + p->off[O_KP]);
  double* f1p = fx ? (double*)(a.ws + p->off[O_F1P]) : nullptr;
  int rc = kf1_pass(p->naux, p->norb, a.ws + p->off[O_B], p->bt,
                    fx ? (double*)(a.ws + p->off[O_W]) : nullptr, kp, f1p, p->kchunks, st, p->ninst,
                    (long long)p->naux * n2, (long long)p->naux * p->norb, (long long)p->kchunks * n2);
  if (rc != NOF_OK) return rc;
  if (fx) {
    rc = reduce_parts(f1p, p->kchunks, n2, p->norb, false, (double*)(a.ws + p->off[O_F1]), st,
                      p->ninst, (long long)p->kchunks * n2, n2);
    if (rc != NOF_OK) return rc;
  }
  return reduce_parts(kp, p->kchunks, n2, p->norb, true, (double*)(a.ws + p->off[O_K]), st,
                      p->ninst, (long long)p->kchunks * n2, n2);
}

int run_f2(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long n2 = (long long)p->norb * p->norb;
  if (p->prec == NOF_P_F64) {
    // F2_i - F1_i = sum_q cK_i[q][s] G_i^q[r][s] - F1_i with the symmetric
    // G_i^q = sum_P b_i^P[q]^T b_i^P[q] of every instance, a chunk of q at a
    // time (instance outer, q inner), each chunk added in q order
    const int gq = exchange_sym_chunk(p->norb, p->ninst);
    double* G = (double*)(a.ws + p->off[O_F2P]);
    const double* b = (const double*)(a.ws + p->off[O_B]);
    const double* F1 = (const double*)(a.ws + p->off[O_F1]);
    double* F = (double*)(a.ws + p->off[O_F2]);
    for (int q0 = 0; q0 < p->norb; q0 += gq) {
      const int qn = std::min(gq, p->norb - q0);
      GemmDesc g{};
      g.M = p->norb; g.N = p->norb; g.K = p->naux;
      g.batch = p->ninst * qn; g.fold = 1; g.binner = qn;
      g.X = b + (long long)q0 * p->norb; g.ldx = n2; g.sx = p->norb; g.sx2 = (long long)p->naux * n2;
      g.x_kmajor = true;
      g.Y = b + (long long)q0 * p->norb; g.ldy = n2; g.sy = p->norb; g.sy2 = (long long)p->naux * n2;
      g.Out = G; g.ldo = p->norb; g.so = n2; g.so2 = (long long)qn * n2;
      g.sym = true;
      g.role = GemmRole::ExchangeFock;
      g.tile = p->tile_f2;
      int rc = gemm_tn(g, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
      if (rc != NOF_OK) return rc;
      rc = exchange_accum(G, qn, p->norb, a.cK + (long long)q0 * p->norb, F1, q0 > 0 ? 1 : 2, F, st,
                          p->ninst, (long long)qn * n2, n2, n2);
      if (rc != NOF_OK) return rc;
    }
    return NOF_OK;
  }
  const int fold = (p->naux + p->f2gpi - 1) / p->f2gpi;
  const int gpi = (p->naux + fold - 1) / fold;
  double* f2p = (double*)(a.ws + p->off[O_F2P]);
  if (fixed_point_plan(p)) {
    // every instance in one launch (cK_i^T in FP32 for each)
    ExDesc e{p->naux, p->norb, fold, (const float*)(a.ws + p->off[O_B]), nullptr, f2p};
    e.ninst = p->ninst;
    e.sb = (long long)p->naux * n2;
    e.so = (long long)gpi * n2;
    e.tile = p->tile_f2;
    const int rc = exchange_fock_fx(e, a.cK, (float*)(a.ws + p->off[O_ST]), st);
    if (rc != NOF_OK) return rc;
    return reduce_parts(f2p, gpi, n2, p->norb, false, (double*)(a.ws + p->off[O_F2]), st, p->ninst,
                        (long long)gpi * n2, n2);
  }
  GemmDesc g{};
  g.M = p->norb; g.N = p->norb; g.K = p->norb;
  g.batch = p->ninst * p->naux; g.fold = fold; g.binner = p->naux;
  g.X = a.ws + p->off[O_B]; g.ldx = p->norb; g.sx = n2; g.sx2 = (long long)p->naux * n2;
  g.x_kmajor = true;
  g.Y = a.ws + p->off[O_B]; g.ldy = p->norb; g.sy = n2; g.sy2 = (long long)p->naux * n2;
  g.S = a.cK; g.lds = p->norb; g.ss2 = n2;
  // partial (instance i, group c) at f2p + (i*gpi + c)*n2: with fold > 1 the
  // epilogue indexes it by group, with fold = 1 by inner*so + outer*so2
  g.Out = f2p; g.ldo = p->norb; g.so = n2; g.so2 = (long long)gpi * n2;
  g.role = GemmRole::ExchangeFock;
  g.tile = p->tile_f2;
  // the Coulomb-type term in the operand loader: the product is F2 - F1
  g.W = (const double*)(a.ws + p->off[O_W]); g.ldw = p->norb; g.sw2 = (long long)p->naux * p->norb;
  int rc = gemm_tn(g, p->bt, p->bt, NOF_F64, p->prec, st);
  if (rc != NOF_OK) return rc;
  return reduce_parts(f2p, gpi, n2, p->norb, false, (double*)(a.ws + p->off[O_F2]), st, p->ninst,
                      (long long)gpi * n2, n2);
}

int run_tail(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long n2 = (long long)p->norb * p->norb;
  const double* h = (const double*)(a.ws + p->off[O_H]);
  const double* F1 = fixed_point_plan(p) ? (const double*)(a.ws + p->off[O_F1]) : nullptr;
  int rc = lambda_grad(p->norb, a.n, h, F1, (double*)(a.ws + p->off[O_F2]), a.lam, a.grad, st,
                       p->ninst, p->norb, n2, n2);
  if (rc != NOF_OK) return rc;
  // energy: h, cJ, cK stride n2 per instance; J, K stride n2
  return energy(p->norb, a.n, h, (double*)(a.ws + p->off[O_J]), (double*)(a.ws + p->off[O_K]),
                a.cJ, a.cK, a.E, (double*)(a.ws + p->off[O_EP]), st, p->ninst, p->norb, n2, n2);
}

int run_iteration(nof_plan_s* p, const Args& a, hipStream_t st) {
  const long long n = (long long)p->ninst * p->nbf * p->norb;
  long long gpk = (n + 255) / 256;
  if (gpk > 4096) gpk = 4096;
  hipLaunchKernelGGL(k_pack_C, dim3((unsigned)gpk), dim3(256), 0, st, p->ninst, p->nbf, p->norb,
                     a.C, (double*)(a.ws + p->off[O_CALL]));
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  if ((rc = run_stage1(p, a, st)) != NOF_OK) return rc;
  if ((rc = run_stage2(p, a, st)) != NOF_OK) return rc;
  if ((rc = run_small(p, a, st)) != NOF_OK) return rc;
  if ((rc = run_pass(p, a, st)) != NOF_OK) return rc;
  if ((rc = run_f2(p, a, st)) != NOF_OK) return rc;
  return run_tail(p, a, st);
}

// Time `reps` launches of one stage; returns milliseconds per launch or -1.
template <class F>
float time_stage(F&& f, hipStream_t st, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.f; }
  float ms = -1.f;
  if (f() == NOF_OK && hipEventRecord(e0, st) == hipSuccess) {
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = f() == NOF_OK;
    if (ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / reps;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}


// ---------------------------------------------------------------------------
// Batched solve: the alternating NO + ON optimisation (the same iteration as
// the single-instance solver) for every instance of a plan at once.  A NO step
// of all instances is one launch sequence (one graph replay when the stream
// can be captured): the batched iteration, max|lambda_i - lambda_i^T|, ADAM on
// the instances still stepping, U_i = exp(y_i), C_i <- C_i U_i.  An instance
// that does not step gets y_i = 0, so U_i = I exactly and C_i is unchanged.
// ---------------------------------------------------------------------------

// max_pq |L_pq - L_qp| of instance blockIdx.x's n x n matrix.
__global__ void k_asym_inst(int n, const double* __restrict__ L, double* __restrict__ out) {
  __shared__ double red[256];
  const long long nn = (long long)n * n;
  L += (long long)blockIdx.x * nn;
  double m = 0.0;
  for (long long i = threadIdx.x; i < nn; i += blockDim.x) {
    const long long p = i / n, q = i - p * n;
    if (q > p) m = fmax(m, fabs(L[p * n + q] - L[q * n + p]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ADAM step of instance blockIdx.y when ctl[3i] != 0 (its sweep runs) and its
// lambda is not yet symmetric (asym[i] > tol); ctl[3i+1], ctl[3i+2] are the
// bias corrections 1 - b1^t, 1 - b2^t of the step it would take.  Other
// instances: y_i = 0, moments unchanged.
__global__ void k_adam_inst(long long n2, const double* __restrict__ g, double* __restrict__ m,
                            double* __restrict__ v, const double* __restrict__ ctl,
                            const double* __restrict__ asym, double tol, double b1, double b2,
                            double lr, double eps, double* __restrict__ y) {
  const int i = blockIdx.y;
  const long long off = (long long)i * n2;
  const bool step = ctl[3 * i] != 0.0 && asym[i] > tol;
  const double c1 = ctl[3 * i + 1], c2 = ctl[3 * i + 2];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n2;
       e += (long long)gridDim.x * blockDim.x) {
    if (!step) {
      y[off + e] = 0.0;
      continue;
    }
    const double gi = g[off + e];
    const double mi = b1 * m[off + e] + (1.0 - b1) * gi;
    const double vi = b2 * v[off + e] + (1.0 - b2) * gi * gi;
    m[off + e] = mi;
    v[off + e] = vi;
    const double mh = mi / c1, vh = vi / c2;
    y[off + e] = -lr * mh / (sqrt(vh) + eps);
  }
}

__global__ void k_copy_f64(long long n, const double* __restrict__ src, double* __restrict__ dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void k_zero_f64(long long n, double* __restrict__ dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = 0.0;
}

unsigned grid_of(long long n) {
  long long g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : g > 4096 ? 4096 : g);
}

// Workspace of the batched solve, after the plan's own.
struct SolveLay {
  size_t n, cJ, cK, lam, grad, m, v, y, U, Cn, E, Eon, asym, orth, ctl, info, act, scr, scr_bytes, total;
};

SolveLay solve_lay(const nof_plan_s* p, int ns, int ng) {
  SolveLay L{};
  const size_t ni = p->ninst, no = p->norb, nb = p->nbf;
  const size_t n2 = no * no * 8;
  size_t o = p->total;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  L.n = take(ni * no * 8);
  L.cJ = take(ni * n2);
  L.cK = take(ni * n2);
  L.lam = take(ni * n2);
  L.grad = take(ni * n2);
  L.m = take(ni * n2);
  L.v = take(ni * n2);
  L.y = take(ni * n2);
  L.U = take(ni * n2);
  L.Cn = take(ni * nb * no * 8);
  L.E = take(ni * 8);
  L.Eon = take(ni * 8);
  L.asym = take(ni * 8);
  L.orth = take(ni * 8);
  L.ctl = take(ni * 3 * 8);
  L.info = take(ni * 3 * sizeof(int));
  L.act = take(ni * sizeof(int));
  size_t s = expm_ws(p->norb, p->ninst);
  s = std::max(s, rotate_ws(p->nbf, p->norb, p->ninst));
  s = std::max(s, ni * occ_ws_stride(p->norb, ns, ng));   // all instances' ON steps at once
  s = std::max(s, orth_ws(p->nbf, p->norb));
  L.scr_bytes = s;
  L.scr = take(s);
  L.total = o;
  return L;
}

struct SolveBufs {
  double *n, *cJ, *cK, *lam, *grad, *m, *v, *y, *U, *Cn, *E, *Eon, *asym, *orth, *ctl;
  int *info, *act;
  void* scr;
  size_t scr_bytes;
};

// One NO step of every instance (see above); ctl must be on the device.
int no_step(nof_plan_s* p, const Args& a, const SolveBufs& w, double* C, const nof_solve_params* prm,
            hipStream_t st) {
  const long long n2 = (long long)p->norb * p->norb;
  const long long cs = (long long)p->nbf * p->norb;
  int rc = run_iteration(p, a, st);
  if (rc != NOF_OK) return rc;
  hipLaunchKernelGGL(k_asym_inst, dim3(p->ninst), dim3(256), 0, st, p->norb, w.lam, w.asym);
  if ((rc = launch_status()) != NOF_OK) return rc;
  hipLaunchKernelGGL(k_adam_inst, dim3(grid_of(n2), p->ninst), dim3(256), 0, st, n2, w.grad, w.m,
                     w.v, w.ctl, w.asym, prm->tol_lambda, prm->beta1, prm->beta2, prm->lr, prm->eps,
                     w.y);
  if ((rc = launch_status()) != NOF_OK) return rc;
  // every instance's exp(y_i) and C_i U_i in the same launches
  if ((rc = expm_antisym(p->norb, w.y, w.U, w.scr, st, p->ninst)) != NOF_OK) return rc;
  if ((rc = rotate_orbitals(p->nbf, p->norb, C, w.U, w.Cn, w.scr, st, p->ninst)) != NOF_OK) return rc;
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_of(cs * p->ninst)), dim3(256), 0, st, cs * p->ninst, w.Cn,
                     C);
  return launch_status();
}

int plan_solve(nof_plan_s* p, const void* B, const double* H, double* C, int ns, int ng,
               const int* members, int map, int func, double* gamma, double* n_out,
               const nof_solve_params* prm, nof_solve_result* res, char* ws, hipStream_t st) {
  const int ni = p->ninst;
  const long long n2 = (long long)p->norb * p->norb;
  const SolveLay L = solve_lay(p, ns, ng);
  SolveBufs w;
  w.n = (double*)(ws + L.n); w.cJ = (double*)(ws + L.cJ); w.cK = (double*)(ws + L.cK);
  w.lam = (double*)(ws + L.lam); w.grad = (double*)(ws + L.grad);
  w.m = (double*)(ws + L.m); w.v = (double*)(ws + L.v); w.y = (double*)(ws + L.y);
  w.U = (double*)(ws + L.U); w.Cn = (double*)(ws + L.Cn);
  w.E = (double*)(ws + L.E); w.Eon = (double*)(ws + L.Eon); w.asym = (double*)(ws + L.asym);
  w.orth = (double*)(ws + L.orth);
  w.ctl = (double*)(ws + L.ctl); w.info = (int*)(ws + L.info); w.act = (int*)(ws + L.act);
  w.scr = ws + L.scr; w.scr_bytes = L.scr_bytes;
  const Args a{B, C, H, w.n, w.cJ, w.cK, w.E, w.lam, w.grad, ws};
  const double* h = (const double*)(ws + p->off[O_H]);
  const double* J = (const double*)(ws + p->off[O_J]);
  const double* K = (const double*)(ws + p->off[O_K]);

  for (int i = 0; i < ni; ++i) {
    res[i] = nof_solve_result{};
    res[i].status = NOF_OK;
  }
  // ADAM moments start at zero; n, cJ, cK are set before their first use but
  // are cleared so that the first integrals pass reads defined values
  int rc = NOF_OK;
  for (double* z : {w.m, w.v, w.cJ, w.cK}) {
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_of(n2 * ni)), dim3(256), 0, st, n2 * ni, z);
    if ((rc = launch_status()) != NOF_OK) return rc;
  }
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_of((long long)ni * p->norb)), dim3(256), 0, st,
                     (long long)ni * p->norb, w.n);
  if ((rc = launch_status()) != NOF_OK) return rc;

  // the NO step as a graph when the stream can be captured
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct GraphGuard {
    hipGraph_t& g;
    hipGraphExec_t& e;
    ~GraphGuard() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } guard{graph, exec};
  if (st != nullptr) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return NOF_E_HIP;
    rc = no_step(p, a, w, C, prm, st);
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != NOF_OK) return rc;
    if (ec != hipSuccess || !graph) return NOF_E_HIP;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) return NOF_E_HIP;
  }

  std::vector<int> live(ni), sweep(ni), tstep(ni, 0), have_prev(ni, 0), hinfo(3 * ni), on_ok(ni, 1);
  std::vector<double> E_prev(ni, 0.0), hE(ni), hA(ni), ctl(3 * ni), hO(ni);
  int failed_status = NOF_OK;
  for (int i = 0; i < ni; ++i) live[i] = 1;
  auto sync = [&]() { return hipStreamSynchronize(st) == hipSuccess ? NOF_OK : NOF_E_HIP; };

  for (int outer = 0; outer < prm->max_outer; ++outer) {
    bool any = false;
    for (int i = 0; i < ni; ++i) any = any || live[i];
    if (!any) break;
    // ON step at fixed orbitals: h_i, J_i, K_i of the current C_i; every
    // running instance in one launch (one workgroup each)
    if ((rc = run_iteration(p, a, st)) != NOF_OK) return rc;
    if (hipMemcpyAsync(w.act, live.data(), ni * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess)
      return NOF_E_HIP;
    rc = occ_batched(ni, w.act, p->norb, ns, ng, members, map, func, h, p->norb + 1, n2, J, K, n2,
                     gamma, w.n, w.Eon, w.info, prm->on_maxit, prm->on_tol, w.scr, st);
    if (rc != NOF_OK) return rc;
    if (hipMemcpyAsync(hinfo.data(), w.info, 3 * ni * sizeof(int), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return NOF_E_HIP;
    if ((rc = sync()) != NOF_OK) return rc;
    for (int i = 0; i < ni; ++i) {
      if (!live[i]) continue;
      if (hinfo[3 * i + 2] != NOF_OK) return hinfo[3 * i + 2];
      if (prm->on_maxit > 0) {
        res[i].on_iters += hinfo[3 * i];
        on_ok[i] = hinfo[3 * i + 1] != 0;
        if (!on_ok[i]) ++res[i].on_unconverged;
      }
      rc = nof_functional_coeffs(p->norb, ns, ng, members, func, w.n + (long long)i * p->norb,
                                 w.cJ + i * n2, w.cK + i * n2, nullptr, w.scr, w.scr_bytes, st);
      if (rc != NOF_OK) return rc;
      sweep[i] = 1;
    }
    // NO sweep at fixed occupations
    for (int t = 0; t < prm->no_steps; ++t) {
      bool stepping = false;
      for (int i = 0; i < ni; ++i) stepping = stepping || sweep[i];
      if (!stepping) break;
      for (int i = 0; i < ni; ++i) {
        const double tt = (double)(tstep[i] + 1);
        ctl[3 * i] = sweep[i] ? 1.0 : 0.0;
        ctl[3 * i + 1] = 1.0 - pow(prm->beta1, tt);
        ctl[3 * i + 2] = 1.0 - pow(prm->beta2, tt);
      }
      if (hipMemcpyAsync(w.ctl, ctl.data(), 3 * ni * sizeof(double), hipMemcpyHostToDevice, st) !=
          hipSuccess)
        return NOF_E_HIP;
      if (exec) {
        if (hipGraphLaunch(exec, st) != hipSuccess) return NOF_E_HIP;
      } else if ((rc = no_step(p, a, w, C, prm, st)) != NOF_OK) {
        return rc;
      }
      if (hipMemcpyAsync(hE.data(), w.E, ni * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(hA.data(), w.asym, ni * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        return NOF_E_HIP;
      if ((rc = sync()) != NOF_OK) return rc;
      for (int i = 0; i < ni; ++i) {
        if (!sweep[i]) continue;
        res[i].E = hE[i];
        res[i].asym = hA[i];
        if (!std::isfinite(hE[i]) || !std::isfinite(hA[i])) {
          // the step was not taken (asym not > tol); the instance stops here
          res[i].status = NOF_E_NOT_CONVERGED;
          failed_status = NOF_E_NOT_CONVERGED;
          sweep[i] = 0;
          live[i] = 0;
        } else if (hA[i] <= prm->tol_lambda) {
          sweep[i] = 0;
        } else {
          ++tstep[i];
          ++res[i].no_steps;
        }
      }
    }
    // orthonormality of each running instance's orbitals after the sweep,
    // repaired past tol_orth
    const long long cs = (long long)p->nbf * p->norb;
    for (int i = 0; i < ni; ++i) {
      if (!live[i]) continue;
      rc = orthonormalize(p->nbf, p->norb, C + i * cs, nullptr, prm->tol_orth, w.orth + i, w.scr, st);
      if (rc != NOF_OK) return rc;
    }
    if (hipMemcpyAsync(hO.data(), w.orth, ni * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
      return NOF_E_HIP;
    if ((rc = sync()) != NOF_OK) return rc;
    for (int i = 0; i < ni; ++i) {
      if (!live[i]) continue;
      res[i].orth = std::max(res[i].orth, hO[i]);
      res[i].outer = outer + 1;
      if (on_ok[i] && res[i].asym <= prm->tol_lambda && have_prev[i] &&
          std::fabs(res[i].E - E_prev[i]) <= prm->tol_energy) {
        res[i].converged = 1;
        live[i] = 0;
        continue;
      }
      E_prev[i] = res[i].E;
      have_prev[i] = 1;
    }
  }
  if (n_out) {
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_of((long long)ni * p->norb)), dim3(256), 0, st,
                       (long long)ni * p->norb, w.n, n_out);
    if ((rc = launch_status()) != NOF_OK) return rc;
  }
  return failed_status;
}
}  // namespace
}  // namespace nof

using namespace nof;

namespace {
template <class F>
int guarded_b(F&& f) {
  try {
    return f();
  } catch (...) {
    return NOF_E_INTERNAL;
  }
}
bool plan_ok(const nof_plan_s* p) { return p != nullptr; }
int f2_target_gpi(const nof_plan_s* p, int tile) {
  const int tn = (p->norb + tile - 1) / tile;
  const long long tiles = (long long)tn * tn * p->ninst;
  long long g = (768 + tiles - 1) / tiles;
  if (g < 1) g = 1;
  if (g > p->naux) g = p->naux;
  return (int)g;
}
}  // namespace

extern "C" {

int nof_plan_create(nof_plan* plan, int ninst, int naux, int nbf, int norb, int prec) {
  return guarded_b([&]() -> int {
    if (!plan) return NOF_E_NULL;
    *plan = nullptr;
    if (ninst < 1 || ninst > 4096 || naux < 1 || nbf < 1 || norb < 1 || naux > (1 << 20) ||
        nbf > (1 << 16) || norb > (1 << 16))
      return NOF_E_DIM;
    if (prec != NOF_P_F64 && prec != NOF_P_F32 && prec != NOF_P_BF16X10 && prec != NOF_P_I8X10)
      return NOF_E_PREC;
    if ((prec == NOF_P_BF16X10 || prec == NOF_P_I8X10) && (long long)ninst * norb > (1 << 20))
      return NOF_E_DIM;
    if (prec == NOF_P_I8X10 && nbf > I8_MAX_K) return NOF_E_DIM;
    nof_plan_s* p = new nof_plan_s();
    p->ninst = ninst; p->naux = naux; p->nbf = nbf; p->norb = norb; p->prec = prec;
    p->bt = prec == NOF_P_F64 ? NOF_F64 : NOF_F32;
    p->tile_s1 = 128; p->tile_s2 = 128; p->tile_f2 = 128;
    p->f2gpi = 1;
    // the exchange partial buffer is sized for the largest split the tuner may pick
    p->kchunks = kf1_parts(naux, norb, ninst, p->bt);
    const int gmax = f2_target_gpi(p, 64) * 4 > naux ? naux : f2_target_gpi(p, 64) * 4;
    p->f2gpi = gmax;
    plan_layout(p);
    p->f2gpi = f2_target_gpi(p, 128);
    p->graph = nullptr; p->exec = nullptr; p->captured = false;
    *plan = p;
    return NOF_OK;
  });
}

size_t nof_plan_ws(nof_plan plan) { return plan_ok(plan) ? plan->total : 0; }

int nof_plan_layout(nof_plan plan, size_t* offsets, size_t* bytes, int max_regions) {
  if (!plan_ok(plan)) return NOF_E_NULL;
  if (max_regions < 0) return NOF_E_ARG;
  const int n = nof::O_N < max_regions ? nof::O_N : max_regions;
  for (int i = 0; i < n; ++i) {
    if (offsets) offsets[i] = plan->off[i];
    if (bytes) bytes[i] = plan->bytes[i];
  }
  return nof::O_N;
}

int nof_plan_get_config(nof_plan plan, int* cfg) {
  if (!plan_ok(plan) || !cfg) return NOF_E_NULL;
  cfg[0] = plan->tile_s1; cfg[1] = plan->tile_s2; cfg[2] = plan->tile_f2; cfg[3] = plan->f2gpi;
  return NOF_OK;
}

int nof_plan_set_config(nof_plan plan, const int* cfg) {
  if (!plan_ok(plan) || !cfg) return NOF_E_NULL;
  for (int i = 0; i < 3; ++i)
    if (cfg[i] != 64 && cfg[i] != 128) return NOF_E_ARG;
  const int gmax = f2_target_gpi(plan, 64) * 4 > plan->naux ? plan->naux : f2_target_gpi(plan, 64) * 4;
  if (cfg[3] < 1 || cfg[3] > gmax) return NOF_E_ARG;
  if (plan->captured) return NOF_E_ARG;
  plan->tile_s1 = cfg[0]; plan->tile_s2 = cfg[1]; plan->tile_f2 = cfg[2]; plan->f2gpi = cfg[3];
  return NOF_OK;
}

#define NOF_PLAN_ARGS_CHECK()                                                            \
  if (!plan_ok(plan)) return NOF_E_NULL;                                                 \
  if (!B || !C || !H || !n || !cJ || !cK || !E || !lambda) return NOF_E_NULL;            \
  if (!ws || ws_bytes < plan->total) return NOF_E_WORKSPACE;

int nof_plan_iteration(nof_plan plan, const void* B, const double* C, const double* H,
                       const double* n, const double* cJ, const double* cK, double* E,
                       double* lambda, double* grad, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
  return guarded_b([&]() -> int {
    NOF_PLAN_ARGS_CHECK();
    Args a{B, C, H, n, cJ, cK, E, lambda, grad, (char*)ws};
    return run_iteration(plan, a, stream);
  });
}

int nof_plan_autotune(nof_plan plan, const void* B, const double* C, const double* H,
                      const double* n, const double* cJ, const double* cK, double* E,
                      double* lambda, double* grad, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  return guarded_b([&]() -> int {
    NOF_PLAN_ARGS_CHECK();
    if (plan->captured) return NOF_E_ARG;
    Args a{B, C, H, n, cJ, cK, E, lambda, grad, (char*)ws};
    int rc = run_iteration(plan, a, stream);        // fills T, b, W with valid data
    if (rc != NOF_OK) return rc;
    const int reps = 3;
    // the INT8 transform stages have one tile shape (128); every other
    // product, the exchange-type term of the INT8 plan included, has two
    const int tiles[2] = {128, 64};
    const int nst = plan->prec == NOF_P_I8X10 ? 1 : 2;
    float best = -1.f;
    int bt1 = plan->tile_s1;
    for (int it = 0; it < nst; ++it) {
      const int t = tiles[it];
      plan->tile_s1 = t;
      const float ms = time_stage([&]() { return run_stage1(plan, a, stream); }, stream, reps);
      if (ms > 0.f && (best < 0.f || ms < best)) { best = ms; bt1 = t; }
    }
    plan->tile_s1 = bt1;
    best = -1.f;
    int bt2 = plan->tile_s2;
    for (int it = 0; it < nst; ++it) {
      const int t = tiles[it];
      plan->tile_s2 = t;
      const float ms = time_stage([&]() { return run_stage2(plan, a, stream); }, stream, reps);
      if (ms > 0.f && (best < 0.f || ms < best)) { best = ms; bt2 = t; }
    }
    plan->tile_s2 = bt2;
    best = -1.f;
    int btf = plan->tile_f2, bg = plan->f2gpi;
    const int gmax = f2_target_gpi(plan, 64) * 4 > plan->naux ? plan->naux : f2_target_gpi(plan, 64) * 4;
    for (int it = 0; it < 2; ++it) {
      const int t = tiles[it];
      const int g0 = f2_target_gpi(plan, t);
      const int cands[3] = {g0 / 2 > 0 ? g0 / 2 : 1, g0, 2 * g0};
      for (int g : cands) {
        if (g > gmax) continue;
        plan->tile_f2 = t;
        plan->f2gpi = g;
        const float ms = time_stage([&]() { return run_f2(plan, a, stream); }, stream, reps);
        if (ms > 0.f && (best < 0.f || ms < best)) { best = ms; btf = t; bg = g; }
      }
    }
    plan->tile_f2 = btf;
    plan->f2gpi = bg;
    // leave the outputs consistent with the chosen configuration
    return run_iteration(plan, a, stream);
  });
}

int nof_plan_capture(nof_plan plan, const void* B, const double* C, const double* H,
                     const double* n, const double* cJ, const double* cK, double* E,
                     double* lambda, double* grad, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  return guarded_b([&]() -> int {
    NOF_PLAN_ARGS_CHECK();
    if (stream == nullptr) return NOF_E_ARG;      // the null stream cannot be captured
    if (plan->captured) {
      (void)hipGraphExecDestroy(plan->exec);
      (void)hipGraphDestroy(plan->graph);
      plan->captured = false;
    }
    Args a{B, C, H, n, cJ, cK, E, lambda, grad, (char*)ws};
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return NOF_E_HIP;
    const int rc = run_iteration(plan, a, stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(stream, &g);
    if (rc != NOF_OK || ec != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != NOF_OK ? rc : NOF_E_HIP;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return NOF_E_HIP;
    }
    plan->graph = g;
    plan->exec = ex;
    plan->captured = true;
    return NOF_OK;
  });
}

int nof_plan_launch(nof_plan plan, hipStream_t stream) {
  if (!plan_ok(plan)) return NOF_E_NULL;
  if (!plan->captured) return NOF_E_ARG;
  return hipGraphLaunch(plan->exec, stream) == hipSuccess ? NOF_OK : NOF_E_HIP;
}

size_t nof_plan_solve_ws(nof_plan plan, int ns, int ng) {
  if (!plan_ok(plan) || ns < 1 || ng < 1 || (long long)ns * (ng + 1) > plan->norb) return 0;
  try {
    return solve_lay(plan, ns, ng).total;
  } catch (...) {
    return 0;
  }
}

int nof_plan_solve(nof_plan plan, const void* B, const double* H, double* C, int ns, int ng,
                   const int* members, int map, int func, double* gamma, double* n_out,
                   const nof_solve_params* p, nof_solve_result* res, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
  return guarded_b([&]() -> int {
    if (!plan_ok(plan)) return NOF_E_NULL;
    if (!B || !H || !C || !members || !gamma || !p || !res) return NOF_E_NULL;
    if (p->max_outer < 1 || p->no_steps < 1 || p->on_maxit < 0 || !(p->lr > 0.0) ||
        !(p->beta1 >= 0.0 && p->beta1 < 1.0) || !(p->beta2 >= 0.0 && p->beta2 < 1.0) ||
        !(p->eps >= 0.0) || !(p->tol_orth >= 0.0) || p->orbopt == 1)
      return NOF_E_ARG;
    const size_t need = nof_plan_solve_ws(plan, ns, ng);
    if (need == 0) return NOF_E_DIM;
    if (!ws || ws_bytes < need) return NOF_E_WORKSPACE;
    return plan_solve(plan, B, H, C, ns, ng, members, map, func, gamma, n_out, p, res, (char*)ws,
                      stream);
  });
}

int nof_plan_destroy(nof_plan plan) {
  if (!plan) return NOF_OK;
  if (plan->captured) {
    (void)hipGraphExecDestroy(plan->exec);
    (void)hipGraphDestroy(plan->graph);
  }
  delete plan;
  return NOF_OK;
}

}  // extern "C"
