// Split-precision BF16 matrix-core contraction (the reduced-precision form of
// the orbital transformation and of the exchange-type generalized-Fock term).
//
//   Out_b[m][n] = sum_k X_b(k, m) * Y_b(k, n) * S(k, n)       (same contract as gemm_tn)
//
// Each FP32/FP64 operand element x is split on load into BF16 pieces
//   x = x0 + x1 + x2 + r,   x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1),
// |r| <= 2^-24 |x| with three pieces (Henry, Tang and Heinecke, "Leveraging the
// bfloat16 artificial intelligence datatype for higher-precision computations",
// ARITH 2019).  Products x_i * y_j of two pieces are exact in FP32; the kernel
// accumulates all pairs with i + j <= ORD:
//   x1:  (0,0)                         NX = NY = 1, ORD = 0
//   x3:  (0,0) (0,1) (1,0)             NX = NY = 2, ORD = 1
//   x6:  (0,0) (0,1) (1,0) (0,2) (1,1) (2,0)   NX = NY = 3, ORD = 2
//   X stored in BF16 (exact as one piece) with a 3-piece Y: (0,0) (0,1) (0,2).
// Products accumulate in FP32 inside one batch (one auxiliary slab) and, when a
// workgroup folds several batches, in FP64 across them.
//
// Layout: 256 threads = 4 waves (2x2), each wave a 64x64 block as 4x4
// fragments of v_mfma_f32_16x16x32_bf16 (lane l holds 8 consecutive k of row
// l%16 at k offset 8*(l/16); output row 4*(l/16)+r, column l%16).  K advances
// 32 per stage.  LDS keeps each piece as [row][k] with k contiguous so a lane
// fetches its 8 values with one 16-byte read; rows are padded to 40 elements
// (80 B) so the 16 lanes of a read phase hit distinct banks.
#include "common.h"

namespace nof {
namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int BM = 128;
constexpr int KT = 32;
constexpr int NTHR = 256;
constexpr int LROW = KT + 8;                 // padded LDS row (bf16 elements)
constexpr int PER_T = KT * BM / NTHR;        // operand elements per thread per stage (16)

__device__ __forceinline__ int xcd_logical(int w, int G) {
  const int q = G >> 3, r = G & 7, x = w & 7, i = w >> 3;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ void upper_tile(int t, int T, int& tm, int& tn) {
  int row = 0;
  while (t >= T - row) { t -= T - row; ++row; }
  tm = row;
  tn = row + t;
}

template <typename T> __device__ __forceinline__ double as_double(T v) { return (double)v; }
template <> __device__ __forceinline__ double as_double<__bf16>(__bf16 v) { return (double)(float)v; }

// Split v into NP bf16 pieces (most significant first).
template <int NP>
__device__ __forceinline__ void split(double v, __bf16 (&p)[3]) {
  const __bf16 h = (__bf16)(float)v;
  p[0] = h;
  if (NP > 1) {
    const double r1 = v - (double)(float)h;
    const __bf16 m = (__bf16)(float)r1;
    p[1] = m;
    if (NP > 2) {
      const double r2 = r1 - (double)(float)m;
      p[2] = (__bf16)(float)r2;
    }
  }
}

template <int NX, int NY, int ORD, typename TX, typename TY, typename TO, bool FLUSH64, bool HAS_S>
__device__ __forceinline__ void bf16_body(const GemmDesc& d, int tiles_n, int ntiles) {
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][NX][BM][LROW];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][NY][BM][LROW];

  if (d.pred && *d.pred <= d.pred_gt) return;
  const int tid = threadIdx.x;
  const int l = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;

  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  const int group = logical / ntiles;
  const int tile = logical - group * ntiles;
  int tm, tn;
  if (d.sym) upper_tile(tile, tiles_n, tm, tn);
  else { tm = tile / tiles_n; tn = tile - tm * tiles_n; }
  const int m0 = tm * BM, n0 = tn * BM;

  const int b_lo = group * d.fold;
  const int b_hi = min(d.batch, b_lo + d.fold);
  const int nkb = (d.K + KT - 1) / KT;
  const int nstage = (b_hi - b_lo) * nkb;

  const TX* __restrict__ X = (const TX*)d.X;
  const TY* __restrict__ Y = (const TY*)d.Y;
  const double* __restrict__ S = d.S;

  // Loader: thread owns column c_t of the tile and k rows kg*16 .. kg*16+15.
  const int c_t = tid & (BM - 1);
  const int kg = tid >> 7;
  const bool xm_ok = m0 + c_t < d.M;
  const bool yn_ok = n0 + c_t < d.N;

  f4v acc[4][4];
  d4v acc64[FLUSH64 ? 4 : 1][FLUSH64 ? 4 : 1];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0, 0, 0, 0};
  if (FLUSH64) {
#pragma unroll
    for (int i = 0; i < (FLUSH64 ? 4 : 1); ++i)
#pragma unroll
      for (int j = 0; j < (FLUSH64 ? 4 : 1); ++j) acc64[i][j] = d4v{0, 0, 0, 0};
  }

  TX xr[PER_T];
  TY yr[PER_T];
  double sr[HAS_S ? PER_T : 1];

  auto load = [&](int s) {
    const int bb = b_lo + s / nkb;
    const int k0 = (s - (bb - b_lo) * nkb) * KT;
    int klim = d.K - k0;
    if (d.Ktot > 0) {
      const long long r = d.Ktot - (long long)bb * d.K - k0;
      if (r < klim) klim = (int)(r < 0 ? 0 : r);
    }
    const int kb = kg * 16;
    const TX* px = X + (long long)bb * d.sx + (long long)(k0 + kb) * d.ldx + (m0 + c_t);
    const TY* py = Y + (long long)bb * d.sy + (long long)(k0 + kb) * d.ldy + (n0 + c_t);
#pragma unroll
    for (int j = 0; j < PER_T; ++j) {
      const bool kin = kb + j < klim;
      xr[j] = (xm_ok && kin) ? px[(long long)j * d.ldx] : (TX)0;
      const bool ok = yn_ok && kin;
      yr[j] = ok ? py[(long long)j * d.ldy] : (TY)0;
      if (HAS_S) sr[HAS_S ? j : 0] = ok ? S[(long long)(k0 + kb + j) * d.lds + (n0 + c_t)] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      bf8v px[3], py[3];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = half * 8 + e;
        __bf16 p[3];
        split<NX>(as_double(xr[j]), p);
#pragma unroll
        for (int q = 0; q < NX; ++q) px[q][e] = p[q];
        const double yv = HAS_S ? as_double(yr[j]) * sr[HAS_S ? j : 0] : as_double(yr[j]);
        split<NY>(yv, p);
#pragma unroll
        for (int q = 0; q < NY; ++q) py[q][e] = p[q];
      }
      const int kofs = kg * 16 + half * 8;
#pragma unroll
      for (int q = 0; q < NX; ++q) *(bf8v*)&Xs[buf][q][c_t][kofs] = px[q];
#pragma unroll
      for (int q = 0; q < NY; ++q) *(bf8v*)&Ys[buf][q][c_t][kofs] = py[q];
    }
  };

  if (nstage > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int kl = 8 * (l >> 4);
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstage) load(s + 1);
    bf8v a[4][NX], bv[4][NY];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < NX; ++q) a[i][q] = *(const bf8v*)&Xs[buf][q][wm * 64 + i * 16 + (l & 15)][kl];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < NY; ++q) bv[j][q] = *(const bf8v*)&Ys[buf][q][wn * 64 + j * 16 + (l & 15)][kl];
    // least significant products first
#pragma unroll
    for (int o = ORD; o >= 0; --o)
#pragma unroll
      for (int px = 0; px < NX; ++px) {
        const int py = o - px;
        if (py < 0 || py >= NY) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][px], bv[j][py], acc[i][j], 0, 0, 0);
      }
    if (FLUSH64 && ((s + 1) % nkb == 0)) {
#pragma unroll
      for (int i = 0; i < (FLUSH64 ? 4 : 1); ++i)
#pragma unroll
        for (int j = 0; j < (FLUSH64 ? 4 : 1); ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = f4v{0, 0, 0, 0};
        }
    }
    if (s + 1 < nstage) store(buf ^ 1);
    __syncthreads();
  }

  TO* __restrict__ Out = (TO*)d.Out;
  const long long ob = (long long)(d.fold == 1 ? b_lo : group) * d.so;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 64 + i * 16 + 4 * (l >> 4) + r;
        const int gn = n0 + wn * 64 + j * 16 + (l & 15);
        double v;
        if (FLUSH64) v = acc64[FLUSH64 ? i : 0][FLUSH64 ? j : 0][r];
        else v = (double)acc[i][j][r];
        if (gm >= d.M || gn >= d.N) continue;
        if (!d.sym) {
          Out[ob + (long long)gm * d.ldo + gn] = (TO)v;
        } else if (gm <= gn) {
          Out[ob + (long long)gm * d.ldo + gn] = (TO)v;
          Out[ob + (long long)gn * d.ldo + gm] = (TO)v;
          if (gm == gn && d.Dg) d.Dg[(long long)b_lo * d.sd + gm] = v;
        }
      }
}

#define NOF_BF16_KERNEL(NAME)                                                                  \
  template <int NX, int NY, int ORD, typename TX, typename TY, typename TO, bool FLUSH64,      \
            bool HAS_S>                                                                        \
  __global__ __launch_bounds__(NTHR, 1) void NAME(GemmDesc d, int tiles_n, int ntiles) {       \
    bf16_body<NX, NY, ORD, TX, TY, TO, FLUSH64, HAS_S>(d, tiles_n, ntiles);                   \
  }
NOF_BF16_KERNEL(k_transform_stage1_bf16)
NOF_BF16_KERNEL(k_transform_stage2_bf16)
NOF_BF16_KERNEL(k_exchange_fock_bf16)
#undef NOF_BF16_KERNEL

template <int NX, int NY, int ORD, typename TX, typename TY, typename TO, bool FLUSH64>
int launch(const GemmDesc& d, hipStream_t st) {
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BM - 1) / BM;
  const int ntiles = d.sym ? tiles_n * (tiles_n + 1) / 2 : tiles_m * tiles_n;
  const int ngroups = (d.batch + d.fold - 1) / d.fold;
  const long long G = (long long)ntiles * ngroups;
  if (G <= 0) return NOF_OK;
  if (G > 0x7fffffffLL) return NOF_E_DIM;
#define NOF_LAUNCH(NAME, HS)                                                                    \
  hipLaunchKernelGGL((NAME<NX, NY, ORD, TX, TY, TO, FLUSH64, HS>), dim3((unsigned)G), dim3(NTHR), \
                     0, st, d, tiles_n, ntiles)
  switch (d.role) {
    case GemmRole::TransformStage1: NOF_LAUNCH(k_transform_stage1_bf16, false); break;
    case GemmRole::TransformStage2: NOF_LAUNCH(k_transform_stage2_bf16, false); break;
    case GemmRole::ExchangeFock:
      if (d.S) NOF_LAUNCH(k_exchange_fock_bf16, true);
      else NOF_LAUNCH(k_exchange_fock_bf16, false);
      break;
    default: return NOF_E_INTERNAL;
  }
#undef NOF_LAUNCH
  return launch_status();
}

template <int NX, int NY, int ORD>
int dispatch_types(const GemmDesc& d, int x_t, int y_t, int out_t, hipStream_t st) {
  const bool flush = d.fold > 1;
  // transform stage 1: X = B (f32 or bf16), Y = C (f64), Out = T (f32)
  if (d.role == GemmRole::TransformStage1 && y_t == NOF_F64 && out_t == NOF_F32 && !flush) {
    if (x_t == NOF_F32) return launch<NX, NY, ORD, float, double, float, false>(d, st);
    return NOF_E_DTYPE;
  }
  // transform stage 2: X = C (f64), Y = T (f32), Out = b (f32)
  if (d.role == GemmRole::TransformStage2 && x_t == NOF_F64 && y_t == NOF_F32 && out_t == NOF_F32 &&
      !flush)
    return launch<NX, NY, ORD, double, float, float, false>(d, st);
  // exchange-type Fock: X = Y = b (f32), Out = FP64 partials
  if (d.role == GemmRole::ExchangeFock && x_t == NOF_F32 && y_t == NOF_F32 && out_t == NOF_F64)
    return flush ? launch<NX, NY, ORD, float, float, double, true>(d, st)
                 : launch<NX, NY, ORD, float, float, double, false>(d, st);
  return NOF_E_DTYPE;
}

}  // namespace

int gemm_bf16(const GemmDesc& d, int x_t, int y_t, int out_t, int prec, hipStream_t st) {
  if (d.sym && d.M != d.N) return NOF_E_DIM;
  if (d.fold < 1 || d.batch < 0) return NOF_E_DIM;
  if (!d.x_kmajor) return NOF_E_DTYPE;
  // B stored in BF16 (exact as one piece) against a three-piece C
  if (x_t == NOF_BF16) {
    if (d.role != GemmRole::TransformStage1 || y_t != NOF_F64 || out_t != NOF_F32 || d.fold > 1)
      return NOF_E_DTYPE;
    if (prec != NOF_P_BF16X6 && prec != NOF_P_BF16X3) return NOF_E_PREC;
    return launch<1, 3, 2, __bf16, double, float, false>(d, st);
  }
  switch (prec) {
    case NOF_P_BF16X1: return dispatch_types<1, 1, 0>(d, x_t, y_t, out_t, st);
    case NOF_P_BF16X3: return dispatch_types<2, 2, 1>(d, x_t, y_t, out_t, st);
    case NOF_P_BF16X6: return dispatch_types<3, 3, 2>(d, x_t, y_t, out_t, st);
    default: return NOF_E_PREC;
  }
}

}  // namespace nof
