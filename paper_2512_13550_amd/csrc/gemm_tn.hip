// Matrix-core contraction used by the orbital transformation (both stages),
// the exchange-type generalized-Fock term and the small J / W products.
//
//   Out_b[m][n] = sum_k X_b(k, m) * Y_b(k, n) * S(k, n)
//
// Both operands are consumed "k-major": a row of the LDS tile is one k and
// holds consecutive m (or n).  That is exactly the layout the 16x16x4 MFMA
// fragments want (lane l takes row k0 + l/16, column l%16), so fragment reads
// are single conflict-free ds_read per lane.  Every operand of this library is
// naturally k-major: B^P (symmetric), C, T^P = B^P C, b^P (symmetric) and D.
//
// Work decomposition: 256 threads = 4 waves in a 2x2 arrangement, each wave
// owns a 64x64 block of the 128x128 output tile as 4x4 MFMA fragments.  K is
// walked in stages of 16 through double-buffered LDS; global loads for stage
// s+1 are in flight while stage s is multiplied.  The batch index (auxiliary
// function P) is the outer grid dimension, remapped so that all tiles of one
// batch run on the same XCD and share its L2.
#include <type_traits>

#include "common.h"

namespace nof {
namespace {

constexpr int KT = 16;             // k per LDS stage
constexpr int NTHR = 256;

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4v acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row (within the 16x16 fragment) held by register r of lane l
  static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef f4v acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// Linear workgroup id -> logical id such that consecutive logical ids share an
// XCD (the dispatcher deals workgroups to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_logical(int w, int G) {
  const int q = G >> 3, r = G & 7, x = w & 7, i = w >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Tile index -> (tm, tn) over the upper triangle tm <= tn of a T x T grid.
__device__ __forceinline__ void upper_tile(int t, int T, int& tm, int& tn) {
  int row = 0;
  while (t >= T - row) { t -= T - row; ++row; }
  tm = row;
  tn = row + t;
}

// FM x FN fragments per wave; the workgroup tile is (32 FM) x (32 FN).
template <typename TC, typename TX, typename TY, typename TO, bool XK, bool FLUSH64, bool HAS_S,
          int FM, int FN>
__device__ __forceinline__ void gemm_body(const GemmDesc& d, int tiles_n, int ntiles) {
  typedef Mfma<TC> MF;
  typedef typename MF::acc_t acc_t;
  constexpr int BMt = 32 * FM, BNt = 32 * FN;
  constexpr int RX = NTHR / BMt, RY = NTHR / BNt;     // k rows per loader pass
  constexpr int PX = KT / RX, PY = KT / RY;           // operand elements per thread
  // padded LDS rows: k and k+1 land on disjoint bank halves
  __shared__ TC Xs[2][KT][BMt + 16];
  __shared__ TC Ys[2][KT][BNt + 16];

  const int tid = threadIdx.x;
  const int l = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;

  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  const int group = logical / ntiles;
  const int tile = logical - group * ntiles;
  int tm, tn;
  if (d.sym) upper_tile(tile, tiles_n, tm, tn);
  else { tm = tile / tiles_n; tn = tile - tm * tiles_n; }
  const int m0 = tm * BMt, n0 = tn * BNt;

  // batches of this group: [b_lo, b_hi) of the inner index, for outer index `outer`
  int outer = 0, b_lo, b_hi;
  if (d.binner > 0) {
    const int gpi = (d.binner + d.fold - 1) / d.fold;
    outer = group / gpi;
    b_lo = (group - outer * gpi) * d.fold;
    b_hi = min(d.binner, b_lo + d.fold);
  } else {
    b_lo = group * d.fold;
    b_hi = min(d.batch, b_lo + d.fold);
  }
  if (d.pred && d.pred[(long long)outer * d.pred_so] <= d.pred_gt) return;
  const long long xo = (long long)outer * d.sx2, yo = (long long)outer * d.sy2;
  const double* __restrict__ Sg = d.S ? d.S + (long long)outer * d.ss2 : nullptr;
  const int nkb = (d.K + KT - 1) / KT;
  const int np = b_hi - b_lo;
  const int nstage = np * nkb;
  // FP64 exchange-type product: the batches (slabs) of the group run inside
  // each k block, so this thread's S values are loaded once per k block and
  // kept while the slabs pass (the accumulation order changes at FP64
  // rounding only; the FP32 form keeps one batch per FP32 sum)
  constexpr bool SREUSE = HAS_S && std::is_same<TC, double>::value;

  const TX* __restrict__ X = (const TX*)d.X + xo;
  const TY* __restrict__ Y = (const TY*)d.Y + yo;
  const double* __restrict__ S = Sg;

  // Stage-invariant part of this thread's load pattern.  Element j of a
  // k-major operand tile is (k = k_t + R j, col = c_t): a wave covers 64
  // consecutive columns of one row.  For an m-major X, element j is
  // (k = tid % 16, m = tid / 16 + 16 j).
  const int cx_t = tid % BMt, kx_t = tid / BMt;
  const int cy_t = tid % BNt, ky_t = tid / BNt;
  const bool xm_ok = XK ? (m0 + cx_t < d.M) : true;
  const bool yn_ok = n0 + cy_t < d.N;
  const int xk_t = tid & (KT - 1), xm_t = tid >> 4;
  // on a diagonal tile of a symmetric product, a wave whose block lies wholly
  // below the diagonal computes nothing that is written: it only loads; a
  // wave on the diagonal skips its fragments below it (i > j)
  const bool lower_wave = d.sym && tm == tn && wm > wn;
  const bool diag_wave = d.sym && tm == tn && wm == wn && FM == FN;

  acc_t acc[FM][FN];
  d4v acc64[FLUSH64 ? FM : 1][FLUSH64 ? FN : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  if (FLUSH64) {
#pragma unroll
    for (int i = 0; i < (FLUSH64 ? FM : 1); ++i)
#pragma unroll
      for (int j = 0; j < (FLUSH64 ? FN : 1); ++j) acc64[i][j] = d4v{0, 0, 0, 0};
  }

  TX xr[PX];
  TY yr[PY];
  // S values kept as loaded (FP64) until the store: converting them at load
  // time would put a wait for every load ahead of the stage's products
  typedef double TS;
  TS sr[HAS_S ? PY : 1];
  // Coulomb-type term folded into the exchange-type product: in the stage
  // whose k rows hold this thread's column n = n0 + cy_t (the lane stages row
  // wk = n - k0 itself), W[b][n] is subtracted from that element after the
  // stores (wdiag: this lane patches in the stage being staged)
  const double* __restrict__ Wg = HAS_S && d.W ? d.W + (long long)outer * d.sw2 : nullptr;
  TS wv = 0;
  int wk = 0;
  bool wdiag = false;

  auto load = [&](int s) {
    const int bb = SREUSE ? b_lo + s % np : b_lo + s / nkb;
    const int k0 = SREUSE ? (s / np) * KT : (s - (bb - b_lo) * nkb) * KT;
    const bool s_new = !SREUSE || s % np == 0;            // S rows of a new k block
    int klim = d.K - k0;                                   // rows of this stage that exist
    if (d.Ktot > 0) {
      const long long r = d.Ktot - (long long)bb * d.K - k0;
      if (r < klim) klim = (int)(r < 0 ? 0 : r);
    }
    if (XK) {
      const TX* px = X + (long long)bb * d.sx + (long long)(k0 + kx_t) * d.ldx + (m0 + cx_t);
#pragma unroll
      for (int j = 0; j < PX; ++j)
        xr[j] = (xm_ok && kx_t + RX * j < klim) ? px[(long long)(RX * j) * d.ldx] : (TX)0;
    } else {
      const TX* px = X + (long long)bb * d.sx + (long long)(m0 + xm_t) * d.ldx + (k0 + xk_t);
      const bool kin = xk_t < klim;
#pragma unroll
      for (int j = 0; j < PX; ++j)
        xr[j] = (kin && m0 + xm_t + 16 * j < d.M) ? px[(long long)(16 * j) * d.ldx] : (TX)0;
    }
    const long long yoff = (long long)(k0 + ky_t) * d.ldy + (n0 + cy_t);
    const TY* py = Y + (long long)bb * d.sy + yoff;
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      const bool ok = yn_ok && ky_t + RY * j < klim;
      yr[j] = ok ? py[(long long)(RY * j) * d.ldy] : (TY)0;
      if (HAS_S && s_new) sr[HAS_S ? j : 0] = ok ? S[(long long)(k0 + ky_t + RY * j) * d.lds + (n0 + cy_t)] : 0.0;
    }
    if (HAS_S) {
      // only stages whose rows [k0, k0 + KT) meet the tile's columns (a
      // workgroup-uniform test) hold diagonal elements
      wdiag = false;
      if (Wg && k0 < n0 + BNt && n0 < k0 + KT) {
        wk = n0 + cy_t - k0;
        wdiag = yn_ok && wk >= 0 && wk < KT && (wk - ky_t) % RY == 0;
        if (wdiag) wv = Wg[(long long)bb * d.ldw + n0 + cy_t];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < PX; ++j) {
      if (XK) Xs[buf][kx_t + RX * j][cx_t] = (TC)xr[j];
      else Xs[buf][xk_t][xm_t + 16 * j] = (TC)xr[j];
    }
#pragma unroll
    for (int j = 0; j < PY; ++j) {
      if (HAS_S) Ys[buf][ky_t + RY * j][cy_t] = (TC)((double)yr[j] * sr[HAS_S ? j : 0]);
      else Ys[buf][ky_t + RY * j][cy_t] = (TC)yr[j];
    }
    // the lane's own diagonal element, written just above (LDS accesses of a
    // wave are ordered)
    if (HAS_S && wdiag) Ys[buf][wk][cy_t] = (TC)((double)Ys[buf][wk][cy_t] - wv);
  };

  if (nstage > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstage) load(s + 1);
    auto products = [&](auto upper_only) {
#pragma unroll
      for (int kk = 0; kk < KT / 4; ++kk) {
        TC a[FM], bv[FN];
        const int kr = kk * 4 + (l >> 4);
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = Xs[buf][kr][wm * 16 * FM + i * 16 + (l & 15)];
#pragma unroll
        for (int j = 0; j < FN; ++j) bv[j] = Ys[buf][kr][wn * 16 * FN + j * 16 + (l & 15)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            if (!decltype(upper_only)::value || i <= j) acc[i][j] = MF::op(a[i], bv[j], acc[i][j]);
      }
    };
    if (diag_wave) products(std::true_type{});
    else if (!lower_wave) products(std::false_type{});
    if (FLUSH64 && ((s + 1) % nkb == 0)) {
      // end of one batch: fold the FP32 partial into FP64
#pragma unroll
      for (int i = 0; i < (FLUSH64 ? FM : 1); ++i)
#pragma unroll
        for (int j = 0; j < (FLUSH64 ? FN : 1); ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = acc_t{0, 0, 0, 0};
        }
    }
    if (s + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }

  // Epilogue
  TO* __restrict__ Out = (TO*)d.Out;
  const long long ob = d.fold == 1 ? (long long)b_lo * d.so + (long long)outer * d.so2
                                   : (long long)group * d.so;
  double* __restrict__ Dg = d.Dg ? d.Dg + (long long)b_lo * d.sd + (long long)outer * d.sd2 : nullptr;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 16 * FM + i * 16 + MF::row(l, r);
        const int gn = n0 + wn * 16 * FN + j * 16 + (l & 15);
        double v;
        if (FLUSH64) v = acc64[FLUSH64 ? i : 0][FLUSH64 ? j : 0][r];
        else v = (double)acc[i][j][r];
        if (gm >= d.M || gn >= d.N) continue;
        if (!d.sym) {
          Out[ob + (long long)gm * d.ldo + gn] = (TO)v;
        } else if (gm <= gn) {
          Out[ob + (long long)gm * d.ldo + gn] = (TO)v;
          Out[ob + (long long)gn * d.ldo + gm] = (TO)v;
          if (gm == gn && Dg) Dg[gm] = v;
        }
      }
}

// One kernel symbol per role, so that profiles attribute time per step.
#define NOF_GEMM_KERNEL(NAME)                                                              \
  template <typename TC, typename TX, typename TY, typename TO, bool XK, bool FLUSH64,     \
            bool HAS_S, int FM, int FN>                                                    \
  __global__ __launch_bounds__(NTHR, 2) void NAME(GemmDesc d, int tiles_n, int ntiles) {   \
    gemm_body<TC, TX, TY, TO, XK, FLUSH64, HAS_S, FM, FN>(d, tiles_n, ntiles);            \
  }
NOF_GEMM_KERNEL(k_transform_stage1)
NOF_GEMM_KERNEL(k_transform_stage2)
NOF_GEMM_KERNEL(k_exchange_fock)
NOF_GEMM_KERNEL(k_gemm_small)
#undef NOF_GEMM_KERNEL

template <typename TC, typename TX, typename TY, typename TO, bool XK, bool FLUSH64, int FM, int FN>
int launch_shape(const GemmDesc& d, hipStream_t st) {
  constexpr int BMt = 32 * FM, BNt = 32 * FN;
  if (d.sym && BMt != BNt) return NOF_E_INTERNAL;
  const int tiles_m = (d.M + BMt - 1) / BMt;
  const int tiles_n = (d.N + BNt - 1) / BNt;
  const int ntiles = d.sym ? tiles_n * (tiles_n + 1) / 2 : tiles_m * tiles_n;
  long long ngroups;
  if (d.binner > 0) {
    if (d.batch % d.binner != 0) return NOF_E_DIM;
    ngroups = (long long)(d.batch / d.binner) * ((d.binner + d.fold - 1) / d.fold);
  } else {
    ngroups = (d.batch + d.fold - 1) / d.fold;
  }
  const long long G = (long long)ntiles * ngroups;
  if (G <= 0) return NOF_OK;
  if (G > 0x7fffffffLL) return NOF_E_DIM;
#define NOF_LAUNCH(NAME)                                                                      \
  do {                                                                                        \
    if (d.S)                                                                                  \
      hipLaunchKernelGGL((NAME<TC, TX, TY, TO, XK, FLUSH64, true, FM, FN>), dim3((unsigned)G), \
                         dim3(NTHR), 0, st, d, tiles_n, ntiles);                              \
    else                                                                                      \
      hipLaunchKernelGGL((NAME<TC, TX, TY, TO, XK, FLUSH64, false, FM, FN>), dim3((unsigned)G), \
                         dim3(NTHR), 0, st, d, tiles_n, ntiles);                              \
  } while (0)
  switch (d.role) {
    case GemmRole::TransformStage1: NOF_LAUNCH(k_transform_stage1); break;
    case GemmRole::TransformStage2: NOF_LAUNCH(k_transform_stage2); break;
    case GemmRole::ExchangeFock: NOF_LAUNCH(k_exchange_fock); break;
    default: NOF_LAUNCH(k_gemm_small); break;
  }
#undef NOF_LAUNCH
  return launch_status();
}

template <typename TC, typename TX, typename TY, typename TO, bool XK, bool FLUSH64>
int launch(const GemmDesc& d, hipStream_t st) {
  if (d.tile == 64) return launch_shape<TC, TX, TY, TO, XK, FLUSH64, 2, 2>(d, st);
  return launch_shape<TC, TX, TY, TO, XK, FLUSH64, 4, 4>(d, st);
}

}  // namespace

int gemm_tn(const GemmDesc& d, int x_t, int y_t, int out_t, int prec, hipStream_t st) {
  if (d.sym && d.M != d.N) return NOF_E_DIM;
  if (d.fold < 1 || d.batch < 0) return NOF_E_DIM;
  if (prec == NOF_P_F64) {
    if (x_t != NOF_F64 || y_t != NOF_F64 || out_t != NOF_F64) return NOF_E_DTYPE;
    return d.x_kmajor ? launch<double, double, double, double, true, false>(d, st)
                      : launch<double, double, double, double, false, false>(d, st);
  }
  if (prec == NOF_P_F32) {
    const bool flush = d.fold > 1;
    if (!d.x_kmajor) return NOF_E_DTYPE;
    if (x_t == NOF_F32 && y_t == NOF_F64 && out_t == NOF_F32 && !flush)
      return launch<float, float, double, float, true, false>(d, st);
    if (x_t == NOF_F64 && y_t == NOF_F32 && out_t == NOF_F32 && !flush)
      return launch<float, double, float, float, true, false>(d, st);
    if (x_t == NOF_F32 && y_t == NOF_F32 && out_t == NOF_F64)
      return flush ? launch<float, float, float, double, true, true>(d, st)
                   : launch<float, float, float, double, true, false>(d, st);
    if (x_t == NOF_F32 && y_t == NOF_F32 && out_t == NOF_F32 && !flush)
      return launch<float, float, float, float, true, false>(d, st);
    return NOF_E_DTYPE;
  }
  return NOF_E_PREC;
}

}  // namespace nof
