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
// x1/x3 accumulate products in FP32 inside one batch (one auxiliary slab) and,
// when a workgroup folds several batches, in FP64 across them; x6 adds every
// 32-deep stage's FP32 partial into FP64 accumulators.  The orbital matrix C
// is split once per call into bf16 planes (k_presplit) stored [piece][col][k],
// so the loaders fill LDS with 16-byte copies.
//
// Layout: 256 threads = 4 waves (2x2), each wave a 64x64 block as 4x4
// fragments of v_mfma_f32_16x16x32_bf16 (lane l holds 8 consecutive k of row
// l%16 at k offset 8*(l/16); output row 4*(l/16)+r, column l%16).  K advances
// 32 per stage.  LDS keeps each piece as [row][k] with k contiguous so a lane
// fetches its 8 values with one 16-byte read; the four 16-byte chunks of a
// row are swizzled (see swz) so that reads and stores are free of bank
// conflicts.
#include "common.h"

namespace nof {
namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int BM = 128;
constexpr int KT = 32;
constexpr int NTHR = 256;
constexpr int LROW = KT;                     // LDS row: 32 bf16 = four 16-byte chunks

// Chunk c of LDS row r sits at position c ^ f(r), f(r) = (r / 2) mod 4
// (element offset returned).  ds_read_b128 serves a wave in four passes of 16
// lanes over 256 bytes of banks (lane quads {0,3,5,6}, {1,2,4,7},
// {8,11,13,14}, {9,10,12,15}) and ds_write_b128 in eight passes of 8
// consecutive lanes over 128 bytes (gfx950, measured with the bank-conflict
// counter): the fragment reads (lane l: row R + l % 16, R a multiple of 16,
// chunk l / 16) and the loader's stores (lane l: row R + l, one chunk) then
// put every pass on distinct 16-byte slots.
__device__ __forceinline__ int swz(int r, int c) { return (c ^ ((r >> 1) & 3)) << 3; }
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

template <typename T> __device__ __forceinline__ float as_float(T v) { return (float)v; }

// Split an FP32 value into NP bf16 pieces (most significant first).  Each
// residual is exact in FP32, and three pieces carry all 24 significand bits.
template <int NP>
__device__ __forceinline__ void split(float v, __bf16 (&p)[3]) {
  const __bf16 h = (__bf16)v;
  p[0] = h;
  if (NP > 1) {
    const float r1 = v - (float)h;
    const __bf16 m = (__bf16)r1;
    p[1] = m;
    if (NP > 2) p[2] = (__bf16)(r1 - (float)m);
  }
}

// Pre-split an FP64 k-major matrix A[k][col] (rows < K, cols < ncol) into NP
// bf16 planes laid out col-major with k contiguous: out[q][col][k], row length
// ldk (a multiple of 32), zero for k >= K.  The pieces are taken from the FP64
// value, so together they carry 24 significant bits of it.
__global__ void k_presplit(const double* __restrict__ A, int K, int ncol, int lda, int ldk, int np,
                           __bf16* __restrict__ out) {
  const long long n = (long long)ncol * ldk;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(i / ldk), k = (int)(i - (long long)col * ldk);
    double v = k < K ? A[(long long)k * lda + col] : 0.0;
    for (int q = 0; q < np; ++q) {
      const __bf16 p = (__bf16)(float)v;
      out[(long long)q * n + i] = p;
      v -= (double)(float)p;
    }
  }
}

// PSX / PSY: the operand is given as pre-split planes (X = planes, ldx = ldk,
// sx = plane stride in elements; see k_presplit).  NBUF: LDS stages (1 or 2).
// A64: every stage's FP32 partial is added into FP64 accumulators (otherwise
// FP32 accumulation spans one batch and FLUSH64 folds batches in FP64).
template <int NX, int NY, int ORD, typename TX, typename TY, typename TO, bool FLUSH64, bool HAS_S,
          bool PSX, bool PSY, int NBUF, bool A64>
__device__ __forceinline__ void bf16_body(const GemmDesc& d, int tiles_n, int ntiles) {
  __shared__ __attribute__((aligned(16))) __bf16 Xs[NBUF][NX][BM][LROW];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[NBUF][NY][BM][LROW];
  constexpr bool ACC2 = FLUSH64 || A64;

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
  d4v acc64[ACC2 ? 4 : 1][ACC2 ? 4 : 1];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0, 0, 0, 0};
  if (ACC2) {
#pragma unroll
    for (int i = 0; i < (ACC2 ? 4 : 1); ++i)
#pragma unroll
      for (int j = 0; j < (ACC2 ? 4 : 1); ++j) acc64[i][j] = d4v{0, 0, 0, 0};
  }

  TX xr[PSX ? 1 : PER_T];
  TY yr[PSY ? 1 : PER_T];
  bf8v xp[PSX ? NX : 1][2], yp[PSY ? NY : 1][2];
  float sr[HAS_S ? PER_T : 1];
  // Coulomb-type term folded in (W given): the element with k == n of the
  // staged rows loses W[b][n] (sk0: first k of the staged rows; sdiag: this
  // lane stages that element)
  const double* __restrict__ Wg = HAS_S ? d.W : nullptr;
  float wv = 0.f;
  int sk0 = 0;
  bool sdiag = false;

  auto load = [&](int s) {
    const int bb = b_lo + s / nkb;
    const int k0 = (s - (bb - b_lo) * nkb) * KT;
    int klim = d.K - k0;
    if (d.Ktot > 0) {
      const long long r = d.Ktot - (long long)bb * d.K - k0;
      if (r < klim) klim = (int)(r < 0 ? 0 : r);
    }
    const int kb = kg * 16;
    if constexpr (PSX) {
      const __bf16* px = (const __bf16*)d.X + (long long)bb * d.sx + (long long)(m0 + c_t) * d.ldx + k0 + kb;
#pragma unroll
      for (int q = 0; q < (PSX ? NX : 1); ++q)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
          xp[q][hh] = xm_ok ? *(const bf8v*)(px + (long long)q * d.psx + 8 * hh) : bf8v{};
    } else {
      const TX* px = X + (long long)bb * d.sx + (long long)(k0 + kb) * d.ldx + (m0 + c_t);
#pragma unroll
      for (int j = 0; j < PER_T; ++j)
        xr[PSX ? 0 : j] = (xm_ok && kb + j < klim) ? px[(long long)j * d.ldx] : (TX)0;
    }
    if constexpr (PSY) {
      const __bf16* py = (const __bf16*)d.Y + (long long)bb * d.sy + (long long)(n0 + c_t) * d.ldy + k0 + kb;
#pragma unroll
      for (int q = 0; q < (PSY ? NY : 1); ++q)
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
          yp[q][hh] = yn_ok ? *(const bf8v*)(py + (long long)q * d.psy + 8 * hh) : bf8v{};
    } else {
      const TY* py = Y + (long long)bb * d.sy + (long long)(k0 + kb) * d.ldy + (n0 + c_t);
#pragma unroll
      for (int j = 0; j < PER_T; ++j) {
        const bool ok = yn_ok && kb + j < klim;
        yr[PSY ? 0 : j] = ok ? py[(long long)j * d.ldy] : (TY)0;
        if (HAS_S) sr[HAS_S ? j : 0] = ok ? (float)S[(long long)(k0 + kb + j) * d.lds + (n0 + c_t)] : 0.f;
      }
    }
    if (HAS_S) {
      sk0 = k0;
      const int dk = n0 + c_t - k0 - kb;
      sdiag = Wg && yn_ok && dk >= 0 && dk < PER_T;
      if (sdiag) wv = (float)Wg[(long long)bb * d.ldw + n0 + c_t];
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int kofs = kg * 16 + half * 8;
      if constexpr (PSX) {
#pragma unroll
        for (int q = 0; q < NX; ++q) *(bf8v*)&Xs[buf][q][c_t][swz(c_t, kofs >> 3)] = xp[PSX ? q : 0][half];
      } else {
        bf8v px[3];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 p[3];
          split<NX>(as_float(xr[PSX ? 0 : half * 8 + e]), p);
#pragma unroll
          for (int q = 0; q < NX; ++q) px[q][e] = p[q];
        }
#pragma unroll
        for (int q = 0; q < NX; ++q) *(bf8v*)&Xs[buf][q][c_t][swz(c_t, kofs >> 3)] = px[q];
      }
      if constexpr (PSY) {
#pragma unroll
        for (int q = 0; q < NY; ++q) *(bf8v*)&Ys[buf][q][c_t][swz(c_t, kofs >> 3)] = yp[PSY ? q : 0][half];
      } else {
        bf8v py[3];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int j = half * 8 + e;
          __bf16 p[3];
          float v = HAS_S ? as_float(yr[PSY ? 0 : j]) * sr[HAS_S ? j : 0] : as_float(yr[PSY ? 0 : j]);
          if (HAS_S && sdiag && sk0 + kg * 16 + j == n0 + c_t) v -= wv;
          split<NY>(v, p);
#pragma unroll
          for (int q = 0; q < NY; ++q) py[q][e] = p[q];
        }
#pragma unroll
        for (int q = 0; q < NY; ++q) *(bf8v*)&Ys[buf][q][c_t][swz(c_t, kofs >> 3)] = py[q];
      }
    }
  };

  if (nstage > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int kl = swz(l & 15, l >> 4);      // fragment rows start at multiples of 16
  for (int s = 0; s < nstage; ++s) {
    const int buf = NBUF == 2 ? (s & 1) : 0;
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
    if (A64 || (FLUSH64 && ((s + 1) % nkb == 0))) {
#pragma unroll
      for (int i = 0; i < (ACC2 ? 4 : 1); ++i)
#pragma unroll
        for (int j = 0; j < (ACC2 ? 4 : 1); ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = f4v{0, 0, 0, 0};
        }
    }
    if (NBUF == 1) __syncthreads();
    if (s + 1 < nstage) store(NBUF == 2 ? (buf ^ 1) : 0);
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
        if (ACC2) v = acc64[ACC2 ? i : 0][ACC2 ? j : 0][r];
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
            bool HAS_S, bool PSX, bool PSY, int NBUF, bool A64>                                \
  __global__ __launch_bounds__(NTHR, (FLUSH64 || A64) ? 1 : 2) void NAME(GemmDesc d, int tiles_n, \
                                                                       int ntiles) {            \
    bf16_body<NX, NY, ORD, TX, TY, TO, FLUSH64, HAS_S, PSX, PSY, NBUF, A64>(d, tiles_n, ntiles); \
  }
NOF_BF16_KERNEL(k_transform_stage1_bf16)
NOF_BF16_KERNEL(k_transform_stage2_bf16)
NOF_BF16_KERNEL(k_exchange_fock_bf16)
#undef NOF_BF16_KERNEL

template <int NX, int NY, int ORD, typename TX, typename TY, typename TO, bool FLUSH64, bool PSX,
          bool PSY, bool A64, int ROLE>
int launch(const GemmDesc& d, hipStream_t st) {
  constexpr int NBUF = (NX + NY) >= 5 ? 1 : 2;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BM - 1) / BM;
  const int ntiles = d.sym ? tiles_n * (tiles_n + 1) / 2 : tiles_m * tiles_n;
  const int ngroups = (d.batch + d.fold - 1) / d.fold;
  const long long G = (long long)ntiles * ngroups;
  if (G <= 0) return NOF_OK;
  if (G > 0x7fffffffLL) return NOF_E_DIM;
  if (ROLE == 1)
    hipLaunchKernelGGL((k_transform_stage1_bf16<NX, NY, ORD, TX, TY, TO, FLUSH64, false, PSX, PSY, NBUF, A64>),
                       dim3((unsigned)G), dim3(NTHR), 0, st, d, tiles_n, ntiles);
  else if (ROLE == 2)
    hipLaunchKernelGGL((k_transform_stage2_bf16<NX, NY, ORD, TX, TY, TO, FLUSH64, false, PSX, PSY, NBUF, A64>),
                       dim3((unsigned)G), dim3(NTHR), 0, st, d, tiles_n, ntiles);
  else
    hipLaunchKernelGGL((k_exchange_fock_bf16<NX, NY, ORD, TX, TY, TO, FLUSH64, true, PSX, PSY, NBUF, A64>),
                       dim3((unsigned)G), dim3(NTHR), 0, st, d, tiles_n, ntiles);
  return launch_status();
}

// x6 accumulates in FP64 every stage; x1 and x3 keep FP32 within a batch.
template <int NX, int NY, int ORD>
int dispatch_types(const GemmDesc& d, int x_t, int y_t, int out_t, hipStream_t st) {
  constexpr bool A64 = ORD >= 2;
  const bool flush = d.fold > 1;
  // transform stage 1: X = B (f32), Y = C pre-split planes, Out = T (f32)
  if (d.role == GemmRole::TransformStage1 && y_t == NOF_BF16 && out_t == NOF_F32 && !flush &&
      x_t == NOF_F32)
    return launch<NX, NY, ORD, float, float, float, false, false, true, A64, 1>(d, st);
  // transform stage 2: X = C pre-split planes, Y = T (f32), Out = b (f32)
  if (d.role == GemmRole::TransformStage2 && x_t == NOF_BF16 && y_t == NOF_F32 && out_t == NOF_F32 &&
      !flush)
    return launch<NX, NY, ORD, float, float, float, false, true, false, A64, 2>(d, st);
  // exchange-type Fock: X = Y = b (f32), S = cK, Out = FP64 partials (x1, x3;
  // x6 takes the x10 element-wise exchange-type product in gemm_fx.hip)
  if constexpr (ORD < 2) {
    if (d.role == GemmRole::ExchangeFock && x_t == NOF_F32 && y_t == NOF_F32 && out_t == NOF_F64 && d.S)
      return flush ? launch<NX, NY, ORD, float, float, double, true, false, false, A64, 3>(d, st)
                   : launch<NX, NY, ORD, float, float, double, false, false, false, A64, 3>(d, st);
  }
  return NOF_E_DTYPE;
}

}  // namespace

int presplit_bf16(const double* A, int K, int ncol, int lda, int ldk, int np, void* out,
                  hipStream_t st) {
  const long long n = (long long)ncol * ldk;
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_presplit, dim3((unsigned)g), dim3(256), 0, st, A, K, ncol, lda, ldk, np,
                     (__bf16*)out);
  return launch_status();
}

int gemm_bf16(const GemmDesc& d, int x_t, int y_t, int out_t, int prec, hipStream_t st) {
  if (d.sym && d.M != d.N) return NOF_E_DIM;
  if (d.fold < 1 || d.batch < 0) return NOF_E_DIM;
  if (!d.x_kmajor || d.Ktot > 0) return NOF_E_DTYPE;
  // B stored in BF16 (exact as one piece) against a three-piece C
  if (x_t == NOF_BF16 && d.role == GemmRole::TransformStage1) {
    if (y_t != NOF_BF16 || out_t != NOF_F32 || d.fold > 1) return NOF_E_DTYPE;
    if (prec != NOF_P_BF16X6 && prec != NOF_P_BF16X3) return NOF_E_PREC;
    return launch<1, 3, 2, __bf16, float, float, false, false, true, true, 1>(d, st);
  }
  switch (prec) {
    case NOF_P_BF16X1: return dispatch_types<1, 1, 0>(d, x_t, y_t, out_t, st);
    case NOF_P_BF16X3: return dispatch_types<2, 2, 1>(d, x_t, y_t, out_t, st);
    case NOF_P_BF16X6: return dispatch_types<3, 3, 2>(d, x_t, y_t, out_t, st);
    // NOF_P_BF16X10 runs in gemm_fx.hip
    default: return NOF_E_PREC;
  }
}

}  // namespace nof
