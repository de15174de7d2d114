// extern "C" entry points declared in include/nof.h: host-side validation,
// workspace layout and the launch sequence of each call.
#include <algorithm>
#include <mutex>
#include <new>

#include "common.h"

using namespace nof;

namespace {

constexpr int kMaxDim = 1 << 20;

bool dim_ok(int x) { return x >= 1 && x <= kMaxDim; }

// The fixed-point forms (BF16 or INT8 pieces): b in FP32, the exchange-type
// term in three element-wise BF16 pieces, the Coulomb-type term from the pass.
bool fixed_point(int prec) { return prec == NOF_P_BF16X10 || prec == NOF_P_I8X10; }
// Forms whose exchange-type product takes no Coulomb-type term: F1 then comes
// from the pass over b (with K) and is subtracted.  X6 shares the x10
// exchange-type product (three element-wise BF16 pieces, six products);
// FP64 takes the exchange-type term through the symmetric per-q products.
bool f1_from_pass(int prec) {
  return fixed_point(prec) || prec == NOF_P_BF16X6 || prec == NOF_P_F64 || prec == NOF_P_F32;
}
// FP64 and FP32 take the exchange-type term through the per-q products G^q
// on the FP64 / FP32 matrix cores (G in FP64).
bool sym_route(int prec) { return prec == NOF_P_F64 || prec == NOF_P_F32; }



// INT8 exchange-type term through the per-q symmetric products while the
// contraction over P stays within the exact int32 depth: per-(q, r) grids
// (norb^2 ints), then for each chunk of q the INT8 planes of the rows
// b^P[q][:] with P contiguous, and the FP64 G^q of the chunk (in the
// partials region); a chunk of planes and G within 4 GiB.
bool i8_sym(int naux) { return naux <= I8_MAX_K; }
int i8_sym_chunk(int naux, int norb) {
  const long long per = 4LL * norb * i8_ldk(naux) + 8LL * norb * norb;
  long long c = (4LL << 30) / per;
  if (c < 1) c = 1;
  if (c > norb) c = norb;
  return (int)c;
}
size_t i8_sym_ws(int naux, int norb) {
  return align256((size_t)norb * norb * sizeof(int)) +
         i8_planes_bytes((long long)i8_sym_chunk(naux, norb) * norb, naux);
}

// Workspace of nof_jk_diag: J split partials, K chunk partials.
struct JkLayout {
  int jsplit, jk, kchunks;
  size_t off_jpart, off_kpart, total;
};
JkLayout jk_layout(int naux, int norb, int bt) {
  JkLayout L;
  const int tn = (norb + 127) / 128;
  const int tiles = tn * (tn + 1) / 2;
  int js = 512 / tiles;
  if (js < 1) js = 1;
  if (js > naux) js = naux;
  L.jk = (naux + js - 1) / js;
  L.jsplit = (naux + L.jk - 1) / L.jk;
  L.kchunks = kf1_parts(naux, norb, 1, bt);
  const size_t n2 = (size_t)norb * norb * sizeof(double);
  L.off_jpart = 0;
  L.off_kpart = align256(L.off_jpart + (size_t)L.jsplit * n2);
  L.total = align256(L.off_kpart + (size_t)L.kchunks * n2);
  return L;
}

// Workspace of nof_gen_fock and nof_fock_terms: W, the partials of the
// Fock-term product (FP64: a chunk of the symmetric products G^q instead) and
// their sum F, the FP32 cK^T of the x10 form, and (the forms whose
// exchange-type product does not take the Coulomb-type term) the F1 chunk
// partials and F1; then (nof_gen_fock) the K chunk partials.
struct FockLayout {
  int kchunks, f2fold, f2groups, gq;
  size_t off_W, off_f2part, off_F, off_St, off_f1part, off_F1, off_i8, terms, off_kpart, total;
};
FockLayout fock_layout(int naux, int norb, int bt, int prec) {
  FockLayout L;
  L.kchunks = kf1_parts(naux, norb, 1, bt);
  const int tn = (norb + 127) / 128;
  const int tiles = tn * tn;
  int groups = (512 + tiles - 1) / tiles;
  if (groups > naux) groups = naux;
  if (groups < 1) groups = 1;
  L.f2fold = (naux + groups - 1) / groups;
  if (prec == NOF_P_I8X10) L.f2fold = i8_exchange_fold(naux, norb);   // exact int32 depth
  L.f2groups = (naux + L.f2fold - 1) / L.f2fold;
  const size_t n2 = (size_t)norb * norb * sizeof(double);
  const bool fx = f1_from_pass(prec);
  const bool i8s = prec == NOF_P_I8X10 && i8_sym(naux);
  L.gq = sym_route(prec) ? exchange_sym_chunk(norb) : i8s ? i8_sym_chunk(naux, norb) : 0;
  L.off_W = 0;
  L.off_f2part = align256((size_t)naux * norb * sizeof(double));
  L.off_F = align256(L.off_f2part + (L.gq > 0 ? (size_t)L.gq : (size_t)L.f2groups) * n2);
  L.off_St = align256(L.off_F + n2);
  L.off_f1part = align256(L.off_St + (size_t)norb * norb * sizeof(float));
  L.off_F1 = align256(L.off_f1part + (fx ? (size_t)L.kchunks * n2 : 0));
  L.off_i8 = align256(L.off_F1 + (fx ? n2 : 0));
  L.terms = align256(L.off_i8 + (i8s ? i8_sym_ws(naux, norb)
                                     : prec == NOF_P_I8X10 ? i8_exchange_ws(1, naux, norb) : 0));
  L.off_kpart = L.terms;
  L.total = align256(L.off_kpart + (size_t)L.kchunks * n2);
  return L;
}

// Workspace of nof_coulomb_fock: W, the F1 and K chunk partials.
struct CoulombLayout {
  int kchunks;
  size_t off_W, off_f1part, off_kpart, total;
};
CoulombLayout coulomb_layout(int naux, int norb, int bt) {
  CoulombLayout L;
  L.kchunks = kf1_parts(naux, norb, 1, bt);
  const size_t n2 = (size_t)norb * norb * sizeof(double);
  L.off_W = 0;
  L.off_f1part = align256((size_t)naux * norb * sizeof(double));
  L.off_kpart = align256(L.off_f1part + (size_t)L.kchunks * n2);
  L.total = align256(L.off_kpart + (size_t)L.kchunks * n2);
  return L;
}

bool prec_ok(int prec) {
  return prec == NOF_P_F64 || prec == NOF_P_F32 || is_bf16_prec(prec) || prec == NOF_P_I8X10;
}

// Storage of b (and of the half-transformed T) for a precision mode.
bool prec_matches(int prec, int t) {
  return (prec == NOF_P_F64 && t == NOF_F64) || (prec == NOF_P_F32 && t == NOF_F32) ||
         ((is_bf16_prec(prec) || prec == NOF_P_I8X10) && t == NOF_F32);
}

// Storage of B for a precision mode: as b, BF16 for the 3-piece split forms,
// fixed-point planes for the two fixed-point forms (the INT8 one only so).
bool b_input_ok(int prec, int Bt) {
  if (Bt == NOF_BF16X4) return prec == NOF_P_BF16X10;
  if (Bt == NOF_I8X4) return prec == NOF_P_I8X10;
  if (prec == NOF_P_I8X10) return false;
  if (prec_matches(prec, Bt)) return true;
  return Bt == NOF_BF16 && (prec == NOF_P_BF16X3 || prec == NOF_P_BF16X6);
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return NOF_E_INTERNAL;
  } catch (...) {
    return NOF_E_INTERNAL;
  }
}

#define NOF_TRY(expr)            \
  do {                           \
    int _rc = (expr);            \
    if (_rc != NOF_OK) return _rc; \
  } while (0)

}  // namespace

extern "C" {

const char* nof_status_str(int status) {
  switch (status) {
    case NOF_OK: return "ok";
    case NOF_E_NULL: return "required pointer is NULL";
    case NOF_E_DIM: return "size out of range or inconsistent";
    case NOF_E_DTYPE: return "unsupported storage type";
    case NOF_E_PREC: return "unsupported precision mode";
    case NOF_E_WORKSPACE: return "workspace missing or too small";
    case NOF_E_HIP: return "HIP runtime call or kernel launch failed";
    case NOF_E_NOT_CONVERGED: return "iteration limit reached before convergence";
    case NOF_E_ARG: return "invalid argument value";
    case NOF_E_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// Bytes of the per-call scratch of one transform stage: the BF16 planes of C
// and, for x10, the grid exponents of the operand split in the loader.
size_t fx_planes_bytes(int nbf, int norb) { return align256((size_t)4 * norb * presplit_ldk(nbf) * 2); }

size_t stage_ws(int naux, int nbf, int norb, int prec, int Bt) {
  if (!is_bf16_prec(prec)) return 256;
  if (prec == NOF_P_BF16X10)
    return fx_planes_bytes(nbf, norb) + align256((size_t)naux * std::max(nbf, norb) * sizeof(int));
  const int np = Bt == NOF_BF16 ? 3 : bf16_pieces(prec);
  return align256((size_t)np * norb * presplit_ldk(nbf) * 2);
}

// Workgroup tile of a batched transform product: 64-wide when 128-wide tiles
// would give fewer than 512 workgroups (the one-electron transform, naux = 1,
// has 16 at Norb = 500), else 128-wide.
int small_grid_tile(int batch, int M, int N, bool sym) {
  const long long tm = (M + 127) / 128, tn = (N + 127) / 128;
  const long long tiles = sym ? tn * (tn + 1) / 2 : tm * tn;
  return tiles * batch < 512 ? 64 : 128;
}

int split_C(int nbf, int norb, const double* C, int prec, int Bt, void* ws, hipStream_t stream) {
  const int np = Bt == NOF_BF16 ? 3 : bf16_pieces(prec);
  return presplit_bf16(C, nbf, norb, norb, (int)presplit_ldk(nbf), np, ws, stream);
}

// Stage 1 of the fixed-point forms may take the rows (P, mu) of all slabs as
// one product: when a slab holds at least one 128-row tile and the rows fit
// int indexing.
bool stage1_fold(int naux, int nbf) { return nbf >= 128 && (long long)naux * nbf + nbf <= 0x7fffffffLL; }

// x10 stage 1 (T^P = B^P C) with the workspace w of one stage: C planes (one
// grid per column), B planes or FP32 B with one grid per row (B^P symmetric:
// row mu = column mu).  With cmax the epilogue also writes the column maxima
// of T per row tile, from which the grid exponents of T's columns (the grids
// of the next stage's split) follow into w after the C planes.
int fx_stage1(int naux, int nbf, int norb, const void* B, int Bt, const double* C, float* T, char* w,
              unsigned* cmax, hipStream_t stream) {
  const long long ldk = presplit_ldk(nbf);
  int* ex = (int*)(w + fx_planes_bytes(nbf, norb));
  NOF_TRY(fx_split_cols(C, nbf, norb, norb, (int)ldk, w, stream));
  FxDesc f{};
  const bool planes = Bt == NOF_BF16X4;
  // planes: the rows (P, mu) of all slabs as one product when a slab holds a
  // whole tile of rows (no slab padded to whole tiles)
  const bool fold = planes && stage1_fold(naux, nbf);
  f.M = fold ? naux * nbf : nbf; f.N = norb; f.K = nbf; f.batch = fold ? 1 : naux;
  f.mslab = fold ? nbf : 0;
  f.X = B;
  if (planes) {
    f.ldx = ldk; f.sx = fold ? 0 : (long long)nbf * ldk; f.psx = (long long)naux * nbf * ldk;
  } else {
    NOF_TRY(fx_row_exps(B, Bt, (long long)naux * nbf, nbf, ex, stream));
    f.ldx = nbf; f.sx = (long long)nbf * nbf; f.ex = ex; f.sex = nbf; f.x_rows = true;
  }
  f.Y = w; f.ldy = ldk; f.sy = 0; f.psy = (long long)norb * ldk;
  f.Out = T; f.ldo = norb; f.so = fold ? 0 : (long long)nbf * norb;
  f.sym = false; f.role = 1;
  f.cmax = cmax; f.scm = (long long)fx_tiles(f.M) * norb;
  NOF_TRY(gemm_fx(f, planes, true, stream));
  if (!cmax) return NOF_OK;
  // the grid exponents of T's columns, per slab, after the C planes in w
  return fx_cmax_exps(cmax, naux, fx_tiles(f.M), norb, (int*)(w + fx_planes_bytes(nbf, norb)), stream, f.mslab,
                      128);
}

// x10 stage 2 (b^P = C^T T^P and D): C planes, T split in the loader on one
// grid per column q of T^P.  grids_ready: the grid exponents are already in
// their slot of w (from the stage-1 column maxima); otherwise a pass over T
// finds them.
int fx_stage2(int naux, int nbf, int norb, const float* T, const double* C, float* b, double* D,
              char* w, bool grids_ready, hipStream_t stream) {
  const long long ldk = presplit_ldk(nbf);
  int* ey = (int*)(w + fx_planes_bytes(nbf, norb));
  NOF_TRY(fx_split_cols(C, nbf, norb, norb, (int)ldk, w, stream));
  if (!grids_ready) NOF_TRY(fx_col_exps(T, naux, nbf, norb, (long long)nbf * norb, ey, stream));
  FxDesc f{};
  f.M = norb; f.N = norb; f.K = nbf; f.batch = naux;
  f.X = w; f.ldx = ldk; f.sx = 0; f.psx = (long long)norb * ldk;
  f.Y = T; f.ldy = norb; f.sy = (long long)nbf * norb; f.ey = ey; f.sey = norb;
  f.Out = b; f.ldo = norb; f.so = (long long)norb * norb;
  f.Dg = D; f.sd = norb; f.sym = true; f.role = 2;
  return gemm_fx(f, true, false, stream);
}

// Column maxima of T per row tile (x10 and INT8, nof_mo_transform only), in
// either stage-1 layout.
size_t fx_cmax_bytes(int naux, int nbf, int norb) {
  long long w = cmax_words(naux, nbf, norb, 128, false);
  if (stage1_fold(naux, nbf)) w = std::max(w, cmax_words(naux, nbf, norb, 128, true));
  return align256((size_t)w * sizeof(unsigned));
}

// INT8 fixed-point transform.  B as written by nof_split_B_i8: planes
// [4][naux*nbf][ldk] and, after them, one grid exponent per row (P, mu).

// Scratch after T: C planes and exponents, the stage-1 column maxima of T,
// the grid exponents of T's columns and T's planes.
struct I8Layout {
  size_t off_Ce, off_cmax, off_Te, off_Tp, total;
};
I8Layout i8_layout(int naux, int nbf, int norb) {
  I8Layout L;
  L.off_Ce = i8_planes_bytes(norb, nbf);
  L.off_cmax = L.off_Ce + align256((size_t)norb * sizeof(int));
  L.off_Te = L.off_cmax + fx_cmax_bytes(naux, nbf, norb);
  L.off_Tp = L.off_Te + align256((size_t)naux * norb * sizeof(int));
  L.total = L.off_Tp + i8_planes_bytes((long long)naux * norb, nbf);
  return L;
}

// b^P = C^T B^P C on the INT8 matrix cores: C split per column; stage 1
// T^P = B^P C (its epilogue gives the column maxima of T); T split per
// column of each T^P on those grids; stage 2 b^P = C^T T^P with D.
int i8_transform(int naux, int nbf, int norb, const void* B, const double* C, float* T, float* b,
                 double* D, char* w, hipStream_t stream) {
  const I8Layout L = i8_layout(naux, nbf, norb);
  const long long ldk = i8_ldk(nbf);
  const unsigned char* Bp = (const unsigned char*)B;
  const int* Be = (const int*)(Bp + i8_planes_bytes((long long)naux * nbf, nbf));
  unsigned char* Cp = (unsigned char*)w;
  int* Ce = (int*)(w + L.off_Ce);
  unsigned* cmax = (unsigned*)(w + L.off_cmax);
  int* Te = (int*)(w + L.off_Te);
  unsigned char* Tp = (unsigned char*)(w + L.off_Tp);
  NOF_TRY(i8_split_cols(C, nbf, norb, norb, (int)ldk, Cp, Ce, stream));
  // the rows (P, mu) of all slabs as one product when a slab holds a whole tile
  const bool fold = stage1_fold(naux, nbf);
  I8Desc f{};
  f.M = fold ? naux * nbf : nbf; f.N = norb; f.K = nbf; f.batch = fold ? 1 : naux;
  f.X = Bp; f.ldx = ldk; f.sx = fold ? 0 : (long long)nbf * ldk; f.psx = (long long)naux * nbf * ldk;
  f.ex = Be; f.sex = fold ? 0 : nbf;
  f.Y = Cp; f.ldy = ldk; f.sy = 0; f.psy = (long long)norb * ldk; f.ey = Ce; f.sey = 0;
  f.Out = T; f.ldo = norb; f.so = fold ? 0 : (long long)nbf * norb;
  f.sym = false; f.role = 1; f.mslab = fold ? nbf : 0;
  f.cmax = cmax; f.scm = (long long)fx_tiles(f.M) * norb;
  NOF_TRY(gemm_i8(f, stream));
  NOF_TRY(i8_cmax_exps(cmax, naux, fx_tiles(f.M), norb, Te, stream, f.mslab));
  NOF_TRY(i8_split_T(T, naux, nbf, norb, (long long)nbf * norb, (int)ldk, Te, Tp, stream));
  I8Desc g{};
  g.M = norb; g.N = norb; g.K = nbf; g.batch = naux;
  g.X = Cp; g.ldx = ldk; g.sx = 0; g.psx = (long long)norb * ldk; g.ex = Ce; g.sex = 0;
  g.Y = Tp; g.ldy = ldk; g.sy = (long long)norb * ldk; g.psy = (long long)naux * norb * ldk;
  g.ey = Te; g.sey = norb;
  g.Out = b; g.ldo = norb; g.so = (long long)norb * norb;
  g.Dg = D; g.sd = norb; g.sym = true; g.role = 2;
  return gemm_i8(g, stream);
}

}  // namespace

extern "C" {

size_t nof_mo_transform_stage_ws(int naux, int nbf, int norb, int prec) {
  if (!dim_ok(naux) || !dim_ok(nbf) || !dim_ok(norb) || !prec_ok(prec)) return 0;
  if (prec == NOF_P_I8X10) return 0;             // nof_mo_transform only
  // B may be given in FP32 or BF16: size for the larger of the two splits of C
  return std::max(stage_ws(naux, nbf, norb, prec, NOF_F32), stage_ws(naux, nbf, norb, prec, NOF_BF16));
}

size_t nof_mo_transform_ws(int naux, int nbf, int norb, int Bt, int bt, int prec) {
  if (!dim_ok(naux) || !dim_ok(nbf) || !dim_ok(norb)) return 0;
  if (!prec_matches(prec, bt) || !b_input_ok(prec, Bt)) return 0;
  if (prec == NOF_P_I8X10)
    return align256((size_t)naux * nbf * norb * sizeof(float)) + i8_layout(naux, nbf, norb).total;
  return align256((size_t)naux * nbf * norb * dtype_size(bt)) + stage_ws(naux, nbf, norb, prec, Bt) +
         (prec == NOF_P_BF16X10 ? fx_cmax_bytes(naux, nbf, norb) : 0);
}

size_t nof_split_B_i8_bytes(int naux, int nbf) {
  if (!dim_ok(naux) || !dim_ok(nbf)) return 0;
  const long long rows = (long long)naux * nbf;
  return i8_planes_bytes(rows, nbf) + align256((size_t)rows * sizeof(int));
}

int nof_split_B_i8(int naux, int nbf, const void* B, int Bt, void* out, size_t out_bytes,
                   hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(nbf)) return NOF_E_DIM;
    if (!B || !out) return NOF_E_NULL;
    if (Bt != NOF_F64 && Bt != NOF_F32) return NOF_E_DTYPE;
    if (out_bytes < nof_split_B_i8_bytes(naux, nbf)) return NOF_E_WORKSPACE;
    const long long rows = (long long)naux * nbf;
    int* e = (int*)((char*)out + i8_planes_bytes(rows, nbf));
    return i8_split_rows(B, Bt, rows, nbf, (int)i8_ldk(nbf), out, e, stream);
  });
}

size_t nof_split_B_bytes(int naux, int nbf) {
  if (!dim_ok(naux) || !dim_ok(nbf)) return 0;
  return (size_t)4 * naux * nbf * presplit_ldk(nbf) * 2;
}

int nof_split_B(int naux, int nbf, const void* B, int Bt, void* planes, size_t planes_bytes,
                hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(nbf)) return NOF_E_DIM;
    if (!B || !planes) return NOF_E_NULL;
    if (Bt != NOF_F64 && Bt != NOF_F32) return NOF_E_DTYPE;
    if (planes_bytes < nof_split_B_bytes(naux, nbf)) return NOF_E_WORKSPACE;
    return fx_split_rows(B, Bt, (long long)naux * nbf, nbf, (int)presplit_ldk(nbf), planes, stream);
  });
}

int nof_mo_transform_stage1(int naux, int nbf, int norb, const void* B, int Bt, const double* C,
                            void* T, int Tt, int prec, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(nbf) || !dim_ok(norb)) return NOF_E_DIM;
    if (!B || !C || !T) return NOF_E_NULL;
    if (dtype_size(Bt) == 0 || dtype_size(Tt) == 0) return NOF_E_DTYPE;
    if (!prec_ok(prec) || prec == NOF_P_I8X10) return NOF_E_PREC;
    if (!prec_matches(prec, Tt)) return NOF_E_PREC;
    if (!b_input_ok(prec, Bt)) return NOF_E_DTYPE;
    const bool bf = is_bf16_prec(prec);
    if (bf && (!ws || ws_bytes < stage_ws(naux, nbf, norb, prec, Bt))) return NOF_E_WORKSPACE;
    if (prec == NOF_P_BF16X10)
      return fx_stage1(naux, nbf, norb, B, Bt, C, (float*)T, (char*)ws, nullptr, stream);
    // T^P[mu][q] = sum_nu B^P[nu][mu] C[nu][q]   (B^P symmetric)
    GemmDesc g1{};
    g1.M = nbf; g1.N = norb; g1.K = nbf; g1.Ktot = 0;
    g1.batch = naux; g1.fold = 1;
    g1.X = B; g1.ldx = nbf; g1.sx = (long long)nbf * nbf; g1.x_kmajor = true;
    g1.Y = C; g1.ldy = norb; g1.sy = 0;
    g1.S = nullptr; g1.lds = 0;
    g1.Out = T; g1.ldo = norb; g1.so = (long long)nbf * norb;
    g1.Dg = nullptr; g1.sd = 0; g1.sym = false;
    // the one-electron transform (naux = 1) is attributed to the small products
    g1.role = naux > 1 ? GemmRole::TransformStage1 : GemmRole::Small;
    g1.tile = small_grid_tile(naux, nbf, norb, false);
    if (!bf) return gemm_tn(g1, Bt, NOF_F64, Tt, prec, stream);
    NOF_TRY(split_C(nbf, norb, C, prec, Bt, ws, stream));
    g1.Y = ws; g1.ldy = presplit_ldk(nbf); g1.psy = (long long)norb * presplit_ldk(nbf);
    return gemm_bf16(g1, Bt, NOF_BF16, Tt, prec, stream);
  });
}

int nof_mo_transform_stage2(int naux, int nbf, int norb, const void* T, int Tt, const double* C,
                            void* b, int bt, double* D, int prec, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(nbf) || !dim_ok(norb)) return NOF_E_DIM;
    if (!T || !C || !b) return NOF_E_NULL;
    if (Tt != bt || dtype_size(bt) == 0 || bt == NOF_BF16) return NOF_E_DTYPE;
    if (!prec_ok(prec) || prec == NOF_P_I8X10) return NOF_E_PREC;
    if (!prec_matches(prec, bt)) return NOF_E_PREC;
    const bool bf = is_bf16_prec(prec);
    if (bf && (!ws || ws_bytes < stage_ws(naux, nbf, norb, prec, NOF_F32))) return NOF_E_WORKSPACE;
    if (prec == NOF_P_BF16X10)
      return fx_stage2(naux, nbf, norb, (const float*)T, C, (float*)b, D, (char*)ws, false, stream);
    // b^P[p][q] = sum_mu C[mu][p] T^P[mu][q], upper tiles + mirror, D
    GemmDesc g2{};
    g2.M = norb; g2.N = norb; g2.K = nbf; g2.Ktot = 0;
    g2.batch = naux; g2.fold = 1;
    g2.X = C; g2.ldx = norb; g2.sx = 0; g2.x_kmajor = true;
    g2.Y = T; g2.ldy = norb; g2.sy = (long long)nbf * norb;
    g2.S = nullptr; g2.lds = 0;
    g2.Out = b; g2.ldo = norb; g2.so = (long long)norb * norb;
    g2.Dg = D; g2.sd = norb; g2.sym = true;
    g2.role = naux > 1 ? GemmRole::TransformStage2 : GemmRole::Small;
    g2.tile = small_grid_tile(naux, norb, norb, true);
    if (!bf) return gemm_tn(g2, NOF_F64, Tt, bt, prec, stream);
    NOF_TRY(split_C(nbf, norb, C, prec, NOF_F32, ws, stream));
    g2.X = ws; g2.ldx = presplit_ldk(nbf); g2.psx = (long long)norb * presplit_ldk(nbf);
    return gemm_bf16(g2, NOF_BF16, Tt, bt, prec, stream);
  });
}

int nof_mo_transform(int naux, int nbf, int norb, const void* B, int Bt, const double* C, void* b,
                     int bt, double* D, int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(nbf) || !dim_ok(norb)) return NOF_E_DIM;
    if (!B || !C || !b) return NOF_E_NULL;
    if (dtype_size(bt) == 0 || dtype_size(Bt) == 0 || bt == NOF_BF16) return NOF_E_DTYPE;
    if (!prec_ok(prec)) return NOF_E_PREC;
    if (!prec_matches(prec, bt)) return NOF_E_PREC;
    if (!b_input_ok(prec, Bt)) return NOF_E_DTYPE;
    const size_t need = nof_mo_transform_ws(naux, nbf, norb, Bt, bt, prec);
    if (!ws || ws_bytes < need) return NOF_E_WORKSPACE;
    const size_t tbytes = align256((size_t)naux * nbf * norb * dtype_size(bt));
    char* sws = (char*)ws + tbytes;
    if (prec == NOF_P_I8X10) return i8_transform(naux, nbf, norb, B, C, (float*)ws, (float*)b, D, sws, stream);
    if (prec == NOF_P_BF16X10) {
      // T, the stage scratch, then the column maxima of T that the stage-1
      // epilogue writes: they give stage 2 its grids without a pass over T
      unsigned* cmax = (unsigned*)(sws + stage_ws(naux, nbf, norb, prec, Bt));
      float* T = (float*)ws;
      NOF_TRY(fx_stage1(naux, nbf, norb, B, Bt, C, T, sws, cmax, stream));
      return fx_stage2(naux, nbf, norb, T, C, (float*)b, D, sws, true, stream);
    }
    const size_t sbytes = ws_bytes - tbytes;
    NOF_TRY(nof_mo_transform_stage1(naux, nbf, norb, B, Bt, C, ws, bt, prec, sws, sbytes, stream));
    return nof_mo_transform_stage2(naux, nbf, norb, ws, bt, C, b, bt, D, prec, sws, sbytes, stream);
  });
}

size_t nof_jk_diag_ws(int naux, int norb, int bt) {
  if (!dim_ok(naux) || !dim_ok(norb)) return 0;
  if (bt != NOF_F64 && bt != NOF_F32) return 0;
  return jk_layout(naux, norb, bt).total;
}

int nof_jk_diag(int naux, int norb, const void* b, int bt, const double* D, double* J, double* K,
                void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(norb)) return NOF_E_DIM;
    if (bt != NOF_F64 && bt != NOF_F32) return NOF_E_DTYPE;
    if ((K && !b) || (J && !D)) return NOF_E_NULL;
    const JkLayout L = jk_layout(naux, norb, bt);
    if (!ws || ws_bytes < L.total) return NOF_E_WORKSPACE;
    char* w = (char*)ws;
    const long long n2 = (long long)norb * norb;
    if (J) {
      double* jpart = (double*)(w + L.off_jpart);
      GemmDesc g{};
      g.M = norb; g.N = norb; g.K = L.jk; g.Ktot = naux;
      g.batch = L.jsplit; g.fold = 1;
      g.X = D; g.ldx = norb; g.sx = (long long)L.jk * norb; g.x_kmajor = true;
      g.Y = D; g.ldy = norb; g.sy = (long long)L.jk * norb;
      g.S = nullptr; g.lds = 0;
      g.Out = jpart; g.ldo = norb; g.so = n2;
      g.Dg = nullptr; g.sd = 0; g.sym = true;
      NOF_TRY(gemm_tn(g, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, stream));
      NOF_TRY(reduce_parts(jpart, L.jsplit, n2, norb, false, J, stream));
    }
    if (K) {
      double* kpart = (double*)(w + L.off_kpart);
      NOF_TRY(kf1_pass(naux, norb, b, bt, nullptr, kpart, nullptr, L.kchunks, stream));
      NOF_TRY(reduce_parts(kpart, L.kchunks, n2, norb, true, K, stream));
    }
    return NOF_OK;
  });
}

}  // extern "C"

namespace {

// FP64 / FP32 exchange-type term through the per-q symmetric products.  b^P
// is symmetric, so
//   F2_rs = sum_P sum_q b^P[r][q] cK[q][s] b^P[q][s] = sum_q cK[q][s] G^q_rs,
//   G^q_rs = sum_P b^P[q][r] b^P[q][s],
// and G^q is symmetric in (r, s): the batched product over q computes the
// upper tiles only (Naux Norb^2 (Norb+1) multiply-adds against 2 Naux Norb^3
// for the product over (P, q)), L.gq values of q at a time into G, each chunk
// then added into F in q order.  With F1, F = F2 - F1.
int exchange_sym(int naux, int norb, const void* b, int bt, const double* cK, const FockLayout& L, double* G,
                 const double* F1, double* F, hipStream_t stream) {
  const size_t es = dtype_size(bt);
  const long long n2 = (long long)norb * norb;
  for (int q0 = 0; q0 < norb; q0 += L.gq) {
    const int qn = std::min(L.gq, norb - q0);
    // G^q = X^T X with X(k = P, m = r) = b^P[q][r]: k-major, P stride norb^2
    GemmDesc g{};
    g.M = norb; g.N = norb; g.K = naux; g.Ktot = 0;
    g.batch = qn; g.fold = 1;
    g.X = (const char*)b + (size_t)q0 * norb * es; g.ldx = n2; g.sx = norb; g.x_kmajor = true;
    g.Y = (const char*)b + (size_t)q0 * norb * es; g.ldy = n2; g.sy = norb;
    g.S = nullptr; g.lds = 0;
    g.Out = G; g.ldo = norb; g.so = n2;
    g.Dg = nullptr; g.sd = 0; g.sym = true;
    g.role = GemmRole::ExchangeFock;
    // FP32: FP32 products and sums over P on the matrix cores, G written in FP64
    NOF_TRY(gemm_tn(g, bt, bt, NOF_F64, bt == NOF_F64 ? NOF_P_F64 : NOF_P_F32, stream));
    const int mode = q0 > 0 ? 1 : (F1 ? 2 : 0);
    NOF_TRY(exchange_accum(G, qn, norb, cK + (long long)q0 * norb, F1, mode, F, stream));
  }
  return NOF_OK;
}

// INT8 exchange-type term through the per-q symmetric products G^q (the
// identity of exchange_sym): every G^q_rs = sum_P b^P[q][r] b^P[q][s] is one
// INT8 fixed-point product over P with one grid per (q, r), exact int32 sums,
// written in FP64 (both triangles of the upper tiles); each chunk of q is
// then added into F2 in q order.  ws: grids, then a chunk of planes.
int i8_exchange_sym(int naux, int norb, const float* b, const double* cK, const FockLayout& L, double* G,
                    char* ws, double* F2, hipStream_t stream) {
  const long long n2 = (long long)norb * norb;
  const long long ldk = i8_ldk(naux);
  int* e = (int*)ws;
  unsigned char* pl = (unsigned char*)(ws + align256((size_t)n2 * sizeof(int)));
  NOF_TRY(i8_slab_grids(b, naux, norb, e, stream));
  for (int q0 = 0; q0 < norb; q0 += L.gq) {
    const int qn = std::min(L.gq, norb - q0);
    // rows b^P[q][:] of the chunk as columns of T_q[k = P][n = r] (row stride norb^2)
    NOF_TRY(i8_split_T(b + (long long)q0 * norb, qn, naux, norb, norb, (int)ldk, e + (long long)q0 * norb, pl,
                       stream, n2));
    I8Desc f{};
    f.M = norb; f.N = norb; f.K = naux; f.batch = qn;
    f.X = pl; f.ldx = ldk; f.sx = norb * ldk; f.psx = (long long)qn * norb * ldk;
    f.ex = e + (long long)q0 * norb; f.sex = norb;
    f.Y = pl; f.ldy = ldk; f.sy = norb * ldk; f.psy = (long long)qn * norb * ldk;
    f.ey = e + (long long)q0 * norb; f.sey = norb;
    f.Out64 = G; f.ldo = norb; f.so = n2;
    f.sym = true; f.role = 3;
    NOF_TRY(gemm_i8(f, stream));
    NOF_TRY(exchange_accum(G, qn, norb, cK + (long long)q0 * norb, nullptr, q0 > 0 ? 1 : 0, F2, stream));
  }
  return NOF_OK;
}

// F2 (exchange-type term) into F2 from the partials in f2part (groups of
// L.f2fold slabs; FP64: a chunk of G); St: norb*norb FP32 scratch of the
// split forms.
int exchange_term(int naux, int norb, const void* b, int bt, const double* cK, const double* W,
                  int prec, const FockLayout& L, double* f2part, float* St, char* i8ws, double* F2,
                  hipStream_t stream) {
  const long long n2 = (long long)norb * norb;
  if (prec == NOF_P_I8X10) {
    if (W) return NOF_E_INTERNAL;
    if (i8_sym(naux)) return i8_exchange_sym(naux, norb, (const float*)b, cK, L, f2part, i8ws, F2, stream);
    // beyond the exact depth: one INT8 product per group of slabs on cK^T in
    // FP32, FP64 partials
    NOF_TRY(fx_transpose(cK, norb, 1, St, stream));
    NOF_TRY(i8_exchange(1, naux, norb, (const float*)b, 0, St, f2part, i8ws, stream));
    return reduce_parts(f2part, L.f2groups, n2, norb, false, F2, stream);
  }
  if (sym_route(prec)) {
    if (W) return NOF_E_INTERNAL;
    return exchange_sym(naux, norb, b, bt, cK, L, f2part, nullptr, F2, stream);
  }
  if (f1_from_pass(prec)) {
    if (W) return NOF_E_INTERNAL;               // this product takes no W (fock_terms)
    ExDesc e{naux, norb, L.f2fold, (const float*)b, nullptr, f2part};
    NOF_TRY(exchange_fock_fx(e, cK, St, stream));
  } else {
    // F2_rs = sum_P sum_q b^P[q][r] (cK[q][s] b^P[q][s])
    GemmDesc g2{};
    g2.M = norb; g2.N = norb; g2.K = norb; g2.Ktot = 0;
    g2.batch = naux; g2.fold = L.f2fold;
    g2.X = b; g2.ldx = norb; g2.sx = n2; g2.x_kmajor = true;
    g2.Y = b; g2.ldy = norb; g2.sy = n2;
    g2.S = cK; g2.lds = norb;
    g2.Out = f2part; g2.ldo = norb; g2.so = n2;
    g2.Dg = nullptr; g2.sd = 0; g2.sym = false;
    g2.role = GemmRole::ExchangeFock;
    g2.W = W; g2.ldw = norb;
    NOF_TRY(gemm_any(g2, bt, bt, NOF_F64, prec, stream));
  }
  return reduce_parts(f2part, L.f2groups, n2, norb, false, F2, stream);
}

// W = D cJ (W[P][s] = sum_q D[P][q] cJ[q][s]), FP64.
int coulomb_weights(int naux, int norb, const double* D, const double* cJ, double* W,
                    hipStream_t stream) {
  GemmDesc gw{};
  gw.M = naux; gw.N = norb; gw.K = norb; gw.Ktot = 0;
  gw.batch = 1; gw.fold = 1;
  gw.X = D; gw.ldx = norb; gw.sx = 0; gw.x_kmajor = false;
  gw.Y = cJ; gw.ldy = norb; gw.sy = 0;
  gw.S = nullptr; gw.lds = 0;
  gw.Out = W; gw.ldo = norb; gw.so = 0;
  gw.Dg = nullptr; gw.sd = 0; gw.sym = false;
  return gemm_tn(gw, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, stream);
}

// F = F2 - F1 = sum_P sum_q b^P[r][q] (cK[q][s] b^P[q][s] - [q == s] W[P][s]).
// x1 / x3: the Coulomb-type term rides in the exchange-type product's operand
// loader.  FP64 and FP32 take the exchange-type term through the symmetric
// per-q products (exchange_sym), the x6 / x10 product stages
// element-wise pieces of FP32 values and the INT8 one fixed-point planes; none
// of these takes it: there F1 comes from the pass over the upper half of b
// (with K when Kpart is given: both from one read of b) and is subtracted.
int fock_terms(int naux, int norb, const void* b, int bt, const double* D, const double* cJ,
               const double* cK, int prec, const FockLayout& L, char* w, double* F,
               double* Kpart, double* K, hipStream_t stream) {
  double* W = (double*)(w + L.off_W);
  NOF_TRY(coulomb_weights(naux, norb, D, cJ, W, stream));
  if (!f1_from_pass(prec))
    return exchange_term(naux, norb, b, bt, cK, W, prec, L, (double*)(w + L.off_f2part),
                         (float*)(w + L.off_St), w + L.off_i8, F, stream);
  const long long n2 = (long long)norb * norb;
  double* f1part = (double*)(w + L.off_f1part);
  double* F1 = (double*)(w + L.off_F1);
  NOF_TRY(kf1_pass(naux, norb, b, bt, W, Kpart, f1part, L.kchunks, stream));
  NOF_TRY(reduce_parts(f1part, L.kchunks, n2, norb, false, F1, stream));
  if (Kpart) NOF_TRY(reduce_parts(Kpart, L.kchunks, n2, norb, true, K, stream));
  if (sym_route(prec))
    return exchange_sym(naux, norb, b, bt, cK, L, (double*)(w + L.off_f2part), F1, F, stream);
  NOF_TRY(exchange_term(naux, norb, b, bt, cK, nullptr, prec, L, (double*)(w + L.off_f2part),
                        (float*)(w + L.off_St), w + L.off_i8, F, stream));
  return subtract(n2, F1, F, stream);
}

}  // namespace

extern "C" {

size_t nof_exchange_fock_ws(int naux, int norb, int bt, int prec) {
  if (!dim_ok(naux) || !dim_ok(norb)) return 0;
  if (!prec_matches(prec, bt)) return 0;
  const FockLayout L = fock_layout(naux, norb, bt, prec);
  return align256((size_t)(L.gq > 0 ? L.gq : L.f2groups) * norb * norb * sizeof(double)) +
         align256((size_t)norb * norb * sizeof(float)) +
         (prec != NOF_P_I8X10 ? 0 : i8_sym(naux) ? i8_sym_ws(naux, norb) : i8_exchange_ws(1, naux, norb));
}

int nof_exchange_fock(int naux, int norb, const void* b, int bt, const double* cK, double* F2,
                      int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(norb)) return NOF_E_DIM;
    if (!b || !cK || !F2) return NOF_E_NULL;
    if (bt != NOF_F64 && bt != NOF_F32) return NOF_E_DTYPE;
    if (!prec_ok(prec)) return NOF_E_PREC;
    if (!prec_matches(prec, bt)) return NOF_E_PREC;
    if (!ws || ws_bytes < nof_exchange_fock_ws(naux, norb, bt, prec)) return NOF_E_WORKSPACE;
    const FockLayout L = fock_layout(naux, norb, bt, prec);
    char* w = (char*)ws;
    double* part = (double*)w;
    float* St = (float*)(w + align256((size_t)(L.gq > 0 ? L.gq : L.f2groups) * norb * norb * sizeof(double)));
    char* i8ws = (char*)St + align256((size_t)norb * norb * sizeof(float));
    return exchange_term(naux, norb, b, bt, cK, nullptr, prec, L, part, St, i8ws, F2, stream);
  });
}

size_t nof_gen_fock_ws(int naux, int norb, int bt, int prec) {
  if (!dim_ok(naux) || !dim_ok(norb)) return 0;
  if (!prec_matches(prec, bt)) return 0;
  return fock_layout(naux, norb, bt, prec).total;
}

int nof_gen_fock(int naux, int norb, const void* b, int bt, const double* D, const double* n,
                 const double* h, const double* cJ, const double* cK, double* lambda, double* grad,
                 double* K_opt, int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(norb)) return NOF_E_DIM;
    if (!b || !D || !n || !h || !cJ || !cK || !lambda) return NOF_E_NULL;
    if (bt != NOF_F64 && bt != NOF_F32) return NOF_E_DTYPE;
    if (!prec_ok(prec)) return NOF_E_PREC;
    if (!prec_matches(prec, bt)) return NOF_E_PREC;
    const FockLayout L = fock_layout(naux, norb, bt, prec);
    if (!ws || ws_bytes < L.total) return NOF_E_WORKSPACE;
    char* w = (char*)ws;
    const long long n2 = (long long)norb * norb;
    double* F = (double*)(w + L.off_F);
    double* kpart = K_opt ? (double*)(w + L.off_kpart) : nullptr;
    const bool fx = f1_from_pass(prec);          // K then comes with F1 from one pass
    NOF_TRY(fock_terms(naux, norb, b, bt, D, cJ, cK, prec, L, w, F, fx ? kpart : nullptr, K_opt,
                       stream));
    if (K_opt && !fx) {
      NOF_TRY(kf1_pass(naux, norb, b, bt, nullptr, kpart, nullptr, L.kchunks, stream));
      NOF_TRY(reduce_parts(kpart, L.kchunks, n2, norb, true, K_opt, stream));
    }
    return lambda_grad(norb, n, h, nullptr, F, lambda, grad, stream);
  });
}

size_t nof_fock_terms_ws(int naux, int norb, int bt, int prec) {
  if (!dim_ok(naux) || !dim_ok(norb)) return 0;
  if (!prec_matches(prec, bt)) return 0;
  return fock_layout(naux, norb, bt, prec).terms;
}

int nof_fock_terms(int naux, int norb, const void* b, int bt, const double* D, const double* cJ,
                   const double* cK, double* F, int prec, void* ws, size_t ws_bytes,
                   hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(norb)) return NOF_E_DIM;
    if (!b || !D || !cJ || !cK || !F) return NOF_E_NULL;
    if (bt != NOF_F64 && bt != NOF_F32) return NOF_E_DTYPE;
    if (!prec_ok(prec)) return NOF_E_PREC;
    if (!prec_matches(prec, bt)) return NOF_E_PREC;
    const FockLayout L = fock_layout(naux, norb, bt, prec);
    if (!ws || ws_bytes < L.terms) return NOF_E_WORKSPACE;
    return fock_terms(naux, norb, b, bt, D, cJ, cK, prec, L, (char*)ws, F, nullptr, nullptr, stream);
  });
}

size_t nof_coulomb_fock_ws(int naux, int norb, int bt) {
  if (!dim_ok(naux) || !dim_ok(norb)) return 0;
  if (bt != NOF_F64 && bt != NOF_F32) return 0;
  return coulomb_layout(naux, norb, bt).total;
}

int nof_coulomb_fock(int naux, int norb, const void* b, int bt, const double* D, const double* cJ,
                     double* F1, double* K_opt, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(naux) || !dim_ok(norb)) return NOF_E_DIM;
    if (!b || !D || !cJ || !F1) return NOF_E_NULL;
    if (bt != NOF_F64 && bt != NOF_F32) return NOF_E_DTYPE;
    const CoulombLayout L = coulomb_layout(naux, norb, bt);
    if (!ws || ws_bytes < L.total) return NOF_E_WORKSPACE;
    char* w = (char*)ws;
    const long long n2 = (long long)norb * norb;
    double* W = (double*)(w + L.off_W);
    double* f1part = (double*)(w + L.off_f1part);
    double* kpart = (double*)(w + L.off_kpart);
    NOF_TRY(coulomb_weights(naux, norb, D, cJ, W, stream));
    NOF_TRY(kf1_pass(naux, norb, b, bt, W, K_opt ? kpart : nullptr, f1part, L.kchunks, stream));
    NOF_TRY(reduce_parts(f1part, L.kchunks, n2, norb, false, F1, stream));
    if (K_opt) NOF_TRY(reduce_parts(kpart, L.kchunks, n2, norb, true, K_opt, stream));
    return NOF_OK;
  });
}

int nof_lambda_grad(int norb, const double* n, const double* h, const double* F1, const double* F2,
                    double* lambda, double* grad, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb)) return NOF_E_DIM;
    if (!n || !h || !F2 || !lambda) return NOF_E_NULL;    // F1 == NULL: F2 is F2 - F1
    return lambda_grad(norb, n, h, F1, F2, lambda, grad, stream);
  });
}

size_t nof_energy_ws(int norb) {
  if (!dim_ok(norb)) return 0;
  return energy_ws(1);
}

int nof_energy(int norb, const double* n, const double* h, const double* J, const double* K,
               const double* cJ, const double* cK, double* E, void* ws, size_t ws_bytes,
               hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb)) return NOF_E_DIM;
    if (!n || !h || !J || !K || !cJ || !cK || !E) return NOF_E_NULL;
    if (!ws || ws_bytes < energy_ws(1)) return NOF_E_WORKSPACE;
    return energy(norb, n, h, J, K, cJ, cK, E, (double*)ws, stream);
  });
}

int nof_coeffs_from_cumulant(int norb, const double* n, const double* Delta, const double* Pi,
                             double* cJ, double* cK, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb)) return NOF_E_DIM;
    if (!n || !Delta || !Pi || !cJ || !cK) return NOF_E_NULL;
    return coeffs_from_cumulant(norb, n, Delta, Pi, cJ, cK, stream);
  });
}

size_t nof_expm_antisym_ws(int norb) {
  if (!dim_ok(norb)) return 0;
  return expm_ws(norb);
}

int nof_expm_antisym(int norb, const double* y, double* U, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb)) return NOF_E_DIM;
    if (!y || !U) return NOF_E_NULL;
    if (!ws || ws_bytes < expm_ws(norb)) return NOF_E_WORKSPACE;
    return expm_antisym(norb, y, U, ws, stream);
  });
}

size_t nof_rotate_orbitals_ws(int nbf, int norb) {
  if (!dim_ok(nbf) || !dim_ok(norb)) return 0;
  return rotate_ws(nbf, norb);
}

int nof_rotate_orbitals(int nbf, int norb, const double* C, const double* U, double* Cout,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(nbf) || !dim_ok(norb)) return NOF_E_DIM;
    if (!C || !U || !Cout) return NOF_E_NULL;
    if (C == Cout) return NOF_E_ARG;
    if (!ws || ws_bytes < rotate_ws(nbf, norb)) return NOF_E_WORKSPACE;
    return rotate_orbitals(nbf, norb, C, U, Cout, ws, stream);
  });
}

size_t nof_orthonormalize_ws(int nbf, int norb) {
  if (!dim_ok(nbf) || !dim_ok(norb)) return 0;
  return orth_ws(nbf, norb);
}

int nof_orthonormalize(int nbf, int norb, double* C, const double* S, double tol, double* err,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(nbf) || !dim_ok(norb)) return NOF_E_DIM;
    if (!C) return NOF_E_NULL;
    if (!(tol >= 0.0)) return NOF_E_ARG;
    if (!ws || ws_bytes < orth_ws(nbf, norb)) return NOF_E_WORKSPACE;
    return orthonormalize(nbf, norb, C, S, tol, err, ws, stream);
  });
}

int nof_adam_step(int norb, const double* g, double* m, double* v, int t, double lr, double beta1,
                  double beta2, double eps, double* y, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb)) return NOF_E_DIM;
    if (!g || !m || !v || !y) return NOF_E_NULL;
    if (t < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
        !(eps >= 0.0))
      return NOF_E_ARG;
    return adam_step(norb, g, m, v, t, lr, beta1, beta2, eps, y, stream);
  });
}

}  // extern "C"

namespace {
bool occ_args_ok(int norb, int ns, int ng, int map, int func) {
  if (!dim_ok(norb) || ns < 1 || ng < 1 || (long long)ns * (ng + 1) > norb) return false;
  if (map != NOF_MAP_TRIG && map != NOF_MAP_SOFTMAX) return false;
  if (func != NOF_FUNC_HF && func != NOF_FUNC_PNOF5 && func != NOF_FUNC_PNOF7) return false;
  return true;
}
}  // namespace

extern "C" {

size_t nof_occ_ws(int norb, int ns, int ng) {
  if (!dim_ok(norb) || ns < 1 || ng < 1 || (long long)ns * (ng + 1) > norb) return 0;
  return occ_ws(norb, ns, ng);
}

int nof_occ_energy_grad(int norb, int ns, int ng, const int* members, int map, int func,
                        const double* gamma, const double* hdiag, int hstride, const double* J,
                        const double* K, double* n, double* E, double* dEdgamma, int* info,
                        void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!occ_args_ok(norb, ns, ng, map, func)) return NOF_E_DIM;
    if (hstride < 1) return NOF_E_ARG;
    if (!members || !gamma || !hdiag || !J || !K) return NOF_E_NULL;
    if (!ws || ws_bytes < occ_ws(norb, ns, ng)) return NOF_E_WORKSPACE;
    return occ_energy_grad(norb, ns, ng, members, map, func, gamma, hdiag, hstride, J, K, n, E,
                           dEdgamma, info, ws, stream);
  });
}

int nof_occ_optimize(int norb, int ns, int ng, const int* members, int map, int func,
                     const double* hdiag, int hstride, const double* J, const double* K,
                     double* gamma, double* n, double* E, int* info, int maxit, double tol,
                     void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!occ_args_ok(norb, ns, ng, map, func)) return NOF_E_DIM;
    if (hstride < 1 || maxit < 0 || !(tol >= 0.0)) return NOF_E_ARG;
    if (!members || !gamma || !hdiag || !J || !K) return NOF_E_NULL;
    if (!ws || ws_bytes < occ_ws(norb, ns, ng)) return NOF_E_WORKSPACE;
    return occ_optimize(norb, ns, ng, members, map, func, hdiag, hstride, J, K, gamma, n, E, info,
                        maxit, tol, ws, stream);
  });
}

}  // extern "C"

namespace {

// Scratch of nof_occ_optimize_noalloc: one array per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel: its
// device address is taken per device with hipGetSymbolAddress on the first
// call made with that device current, and kept.
constexpr size_t kOccScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kOccScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

int occ_scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return NOF_E_HIP;
  if (dev < 0 || dev >= kScratchDevices) return NOF_E_INTERNAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NOF_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NOF_OK;
}

}  // namespace

extern "C" {

int nof_occ_optimize_noalloc(int norb, int ns, int ng, const int* members, int map, int func,
                             const double* hdiag, int hstride, const double* J, const double* K,
                             double* gamma, double* n, double* E, int* info, int maxit, double tol,
                             hipStream_t stream) {
  return guarded([&]() -> int {
    if (!occ_args_ok(norb, ns, ng, map, func)) return NOF_E_DIM;
    if (hstride < 1 || maxit < 0 || !(tol >= 0.0)) return NOF_E_ARG;
    if (!members || !gamma || !hdiag || !J || !K) return NOF_E_NULL;
    if (occ_ws(norb, ns, ng) > kOccScratchBytes) return NOF_E_DIM;
    void* ws = nullptr;
    NOF_TRY(occ_scratch_of_current_device(&ws));
    return occ_optimize(norb, ns, ng, members, map, func, hdiag, hstride, J, K, gamma, n, E, info,
                        maxit, tol, ws, stream);
  });
}

int nof_functional_coeffs(int norb, int ns, int ng, const int* members, int func, const double* n,
                          double* cJ, double* cK, int* info, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  return guarded([&]() -> int {
    if (!occ_args_ok(norb, ns, ng, NOF_MAP_TRIG, func)) return NOF_E_DIM;
    if (!members || !n || !cJ || !cK) return NOF_E_NULL;
    if (!ws || ws_bytes < occ_ws(norb, ns, ng)) return NOF_E_WORKSPACE;
    return functional_coeffs(norb, ns, ng, members, func, n, cJ, cK, ws, info, stream);
  });
}

int nof_mlp_nparams(void) { return mlp_nparams(); }

int nof_mlp_targets(int n, const double* occ, float* theta, hipStream_t stream) {
  return guarded([&]() -> int {
    if (n < 1) return NOF_E_DIM;
    if (!occ || !theta) return NOF_E_NULL;
    return mlp_targets(n, occ, theta, stream);
  });
}

size_t nof_mlp_ws(int rows) {
  if (rows < 1) return 0;
  return mlp_ws(rows);
}

size_t nof_mlp_features_ws(int norb) {
  if (!dim_ok(norb)) return 0;
  return align256((size_t)norb * 5 * sizeof(double));
}

int nof_mlp_features(int norb, const double* hdiag, int hstride, const double* J, const double* K,
                     float* X, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb)) return NOF_E_DIM;
    if (hstride < 1) return NOF_E_ARG;
    if (!hdiag || !J || !K || !X) return NOF_E_NULL;
    if (!ws || ws_bytes < nof_mlp_features_ws(norb)) return NOF_E_WORKSPACE;
    return mlp_features(norb, hdiag, hstride, J, K, X, ws, stream);
  });
}

int nof_mlp_forward(int rows, const float* X, const float* params, float* theta,
                    hipStream_t stream) {
  return guarded([&]() -> int {
    if (rows < 1 || rows > (1 << 28)) return NOF_E_DIM;
    if (!X || !params || !theta) return NOF_E_NULL;
    return mlp_forward(rows, X, params, theta, stream);
  });
}

int nof_mlp_loss_grad(int rows, const float* X, const float* target, const float* params,
                      float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    if (rows < 1 || rows > (1 << 28)) return NOF_E_DIM;
    if (!X || !target || !params || !grad) return NOF_E_NULL;
    if (!ws || ws_bytes < mlp_ws(rows)) return NOF_E_WORKSPACE;
    return mlp_loss_grad(rows, X, target, params, grad, loss, ws, stream);
  });
}

int nof_mlp_adam(int nparams, float* params, const float* grad, float* m, float* v, int t,
                 float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  return guarded([&]() -> int {
    if (nparams < 1) return NOF_E_DIM;
    if (!params || !grad || !m || !v) return NOF_E_NULL;
    if (t < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
      return NOF_E_ARG;
    return mlp_adam(nparams, params, grad, m, v, t, lr, beta1, beta2, eps, stream);
  });
}

int nof_mlp_warm_gamma(int norb, int ns, int ng, const int* members, int map, const float* theta,
                       double nfloor, double* gamma, int* info, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!dim_ok(norb) || ns < 1 || ng < 1 || ng > 64 || (long long)ns * (ng + 1) > norb)
      return NOF_E_DIM;
    if (map != NOF_MAP_TRIG && map != NOF_MAP_SOFTMAX) return NOF_E_ARG;
    if (!(nfloor >= 0.0 && nfloor < 1.0 / (ng + 1))) return NOF_E_ARG;
    if (!members || !theta || !gamma) return NOF_E_NULL;
    return mlp_warm_gamma(norb, ns, ng, members, map, theta, nfloor, gamma, info, stream);
  });
}

}  // extern "C"
