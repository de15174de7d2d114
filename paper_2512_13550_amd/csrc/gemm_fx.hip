// Fixed-point split-precision transform (the NOF_P_BF16X10 form of the two
// stages of the orbital transformation, b^P = C^T B^P C).
//
//   Out_b[m][n] = sum_k X_b(k, m) * Y_b(k, n)
//
// The matrix cores add the 32 products of one BF16 instruction with a
// datapath aligned to the largest term, so element-wise BF16 pieces (x6) do
// not sum correctly rounded and cancellation leaves errors of many ulps of
// the result.  Here every row m of X and every column n of Y gets one grid
// over the whole contraction: with 2^E above its largest magnitude,
//   x = sum_{q<4} n_q 2^(E-7-8q) + r,   n_q integers, |n_q| <= 128,
//   |r| <= 2^(E-32)
// (Ozaki, Ogita, Oishi and Rump, "Error-free transformations of matrix
// multiplication by using fast routines of matrix multiplication", Numer.
// Algorithms 2012, with BF16 pieces; each n_q 2^(...) is exact in BF16).  The
// order-0 products n_0 n_0' are integers of at most 2^14 units of
// 2^(Ex+Ey-14), so up to K = 1024 their running sum (<= 2^24 units) is exact
// in FP32: it has its own accumulator.  Orders 1..3 (2^-8 and less of the
// result) share a second FP32 accumulator.  The ten products of order <= 3
// leave a truncation of order 2^-32 of |x||y|.  For K > 1024 the order-0 sum
// is added to FP64 every 1024 terms (BIGK variant).
//
// Layout: the workgroup tile is TS x TS with two rows of waves, each wave
// TS/2 x 32 as fragments of v_mfma_f32_16x16x32_bf16 (lane l holds 8
// consecutive k of row l%16 at k offset 8*(l/16); output row 4*(l/16)+r,
// column l%16): TS = 128 is 512 threads = 8 waves (2 x 4), one workgroup per
// CU; TS = 64 (for matrices of a few hundred rows, where 128-wide tiles would
// be mostly padding) is 256 threads = 4 waves (2 x 2), two workgroups per
// CU.  Each output element is summed in the same order either way, so the
// two shapes give identical results.  LDS holds the four pieces as [row][k]
// (k in swizzled 16-byte chunks, see swz), in two buffers: the next stage is
// stored while the current one is multiplied.  The operand split in a loader
// (a row of X or column of Y) is shared by TS output columns/rows.
//
// Operands are either pre-split planes (X: [4][..][m][ldk], k contiguous) or
// FP32 values split in the loader against per-row / per-column grid
// exponents computed by a pass before the product.
#include "common.h"

namespace nof {
namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int KT = 32;
// Workgroup shape of a TS x TS tile (TS = 128 or 64): NT threads, WN waves
// along the columns (32 columns each), two along the rows (WR rows each, FM
// fragments of 16), MINB workgroups per CU.
template <int TS>
struct Tile {
  static_assert(TS == 128 || TS == 64, "tile edge");
  static constexpr int NT = 4 * TS;
  static constexpr int WN = TS / 32;
  static constexpr int WR = TS / 2;
  static constexpr int FM = WR / 16;
  static constexpr int MINB = TS == 128 ? 1 : 2;
};
constexpr int EXACT_K = 1024;           // order-0 sums stay exact in FP32 up to this depth
constexpr int EMIN = -90, EMAX = 128;   // grid exponent range (all scales normal FP32)

__device__ __forceinline__ int xcd_logical(int w, int G) {
  const int q = G >> 3, r = G & 7, x = w & 7, i = w >> 3;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ float pow2f(int e) { return __int_as_float((127 + e) << 23); }

__device__ __forceinline__ int clamp_exp(int e) { return e < EMIN ? EMIN : (e > EMAX ? EMAX : e); }

// Smallest E with 2^E > m, from the bits of a non-negative FP32 m.
__device__ __forceinline__ int grid_exp_bits(unsigned mbits) {
  return clamp_exp((int)(mbits >> 23) - 126);
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// Four pieces of each of two values on the grid of exponent E (|v| < 2^E):
// n_q 2^(E-7-8q) with n_q = rint of what the previous pieces left; each piece
// pair is one packed BF16 conversion (exact: |n_q| <= 128).
__device__ __forceinline__ void split_g2(f2v v, int E, bf2v (&p)[4]) {
  f2v t = v * pow2f(7 - E);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f2v n = {rintf(t[0]), rintf(t[1])};
    p[q] = __builtin_convertvector(n * pow2f(E - 7 - 8 * q), bf2v);
    t = (t - n) * 256.0f;
  }
}

__device__ __forceinline__ void split_g64(double v, int E, __bf16 (&p)[4]) {
  double t = ldexp(v, 7 - E);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double n = rint(t);
    p[q] = (__bf16)(float)ldexp(n, E - 7 - 8 * q);
    t = (t - n) * 256.0;
  }
}

// Grid exponents of the rows of A[nrow][K] (rows contiguous): one wave per row.
template <typename T>
__global__ void k_row_exps(const T* __restrict__ A, long long nrow, int K, int* __restrict__ e) {
  const int l = threadIdx.x & 63;
  const long long wpb = blockDim.x >> 6;
  for (long long row = blockIdx.x * wpb + (threadIdx.x >> 6); row < nrow; row += (long long)gridDim.x * wpb) {
    const T* a = A + row * K;
    double m = 0.0;
    for (int k = l; k < K; k += 64) m = fmax(m, fabs((double)a[k]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (l == 0) {
      int E;
      frexp(m, &E);
      e[row] = clamp_exp(E);
    }
  }
}

// Grid exponents of the columns of A_b[K][N] (FP32, batch stride sa):
// e[b*N + n] from max_k |A_b[k][n]|.  Block: 64 columns x 4 row groups (lanes
// along n read contiguous rows), combined through LDS.
__global__ void k_col_exps(const float* __restrict__ A, int batch, int K, int N, long long sa,
                           int* __restrict__ e) {
  __shared__ unsigned red[4][64];
  const int cb = (N + 63) / 64;
  const int c = threadIdx.x & 63, kg = threadIdx.x >> 6;
  for (long long blk = blockIdx.x; blk < (long long)batch * cb; blk += gridDim.x) {
    const long long b = blk / cb;
    const int n = (int)(blk - b * cb) * 64 + c;
    unsigned m = 0;
    if (n < N) {
      const float* a = A + b * sa + n;
#pragma unroll 4
      for (int k = kg; k < K; k += 4) m = max(m, __float_as_uint(a[(long long)k * N]) & 0x7fffffffu);
    }
    red[kg][c] = m;
    __syncthreads();
    if (kg == 0 && n < N) e[b * N + n] = grid_exp_bits(max(max(red[0][c], red[1][c]), max(red[2][c], red[3][c])));
    __syncthreads();
  }
}

// Grid exponents of the columns of T_b from the per-row-tile column maxima
// that the stage-1 epilogue wrote: e[b*N + n] from max_t cmax[b][t][n], or
// (mslab > 0) from the folded layout (slab_cmax).
__global__ void k_cmax_exps(const unsigned* __restrict__ cmax, long long batch, int tiles, int N,
                            int* __restrict__ e, int mslab, int ts) {
  const long long total = batch * N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long b = i / N;
    const int n = (int)(i - b * N);
    unsigned m = 0;
    if (mslab > 0) {
      m = slab_cmax(cmax, b, mslab, ts, tiles, N, n);
    } else {
      const unsigned* c = cmax + b * tiles * N + n;
      for (int t = 0; t < tiles; ++t) m = max(m, c[(long long)t * N]);
    }
    e[i] = grid_exp_bits(m);
  }
}

// Planes of the columns of an FP64 k-major matrix A[k][col] (k < K):
// out[q][col][ldk], one grid per column.  Block: 16 columns; the column
// maxima from 16 row groups, then each wave splits four columns with lanes
// along k (contiguous plane writes).
__global__ void k_split_cols(const double* __restrict__ A, int K, int ncol, int lda, int ldk,
                             __bf16* __restrict__ out) {
  __shared__ double red[16][16];
  __shared__ int ecol[16];
  const long long plane = (long long)ncol * ldk;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int c = t & 15, kg = t >> 4;
  for (int c0 = blockIdx.x * 16; c0 < ncol; c0 += gridDim.x * 16) {
    double m = 0.0;
    if (c0 + c < ncol)
      for (int k = kg; k < K; k += 16) m = fmax(m, fabs(A[(long long)k * lda + c0 + c]));
    red[kg][c] = m;
    __syncthreads();
    if (kg == 0) {
      double mm = 0.0;
      for (int i = 0; i < 16; ++i) mm = fmax(mm, red[i][c]);
      int E;
      frexp(mm, &E);
      ecol[c] = clamp_exp(E);
    }
    __syncthreads();
    for (int cc = 4 * w; cc < 4 * w + 4; ++cc) {
      const int col = c0 + cc;
      if (col >= ncol) break;
      __bf16* o = out + (long long)col * ldk;
      for (int k = l; k < ldk; k += 64) {
        __bf16 p[4];
        split_g64(k < K ? A[(long long)k * lda + col] : 0.0, ecol[cc], p);
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q * plane + k] = p[q];
      }
    }
    __syncthreads();
  }
}

// Planes of the rows of A[nrow][K] (FP64 or FP32, rows contiguous):
// out[q][row][ldk], one grid per row; one wave per row.
template <typename T>
__global__ void k_split_rows(const T* __restrict__ A, long long nrow, int K, int ldk,
                             __bf16* __restrict__ out) {
  const int l = threadIdx.x & 63;
  const long long wpb = blockDim.x >> 6;
  const long long plane = nrow * ldk;
  for (long long row = blockIdx.x * wpb + (threadIdx.x >> 6); row < nrow; row += (long long)gridDim.x * wpb) {
    const T* a = A + row * K;
    double m = 0.0;
    for (int k = l; k < K; k += 64) m = fmax(m, fabs((double)a[k]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    int E;
    frexp(m, &E);
    E = clamp_exp(E);
    for (int k = l; k < ldk; k += 64) {
      __bf16 p[4];
      split_g64(k < K ? (double)a[k] : 0.0, E, p);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q * plane + row * ldk + k] = p[q];
    }
  }
}

// LDS rows hold the 32 k of one stage as four 16-byte chunks, chunk c of row
// r at position c ^ f(r), f(r) = (r / 2) mod 4.  On gfx950 (measured with the
// bank-conflict counter over lane-address patterns) ds_read_b128 serves a
// wave in four passes of 16 lanes over 256 bytes of banks, a pass taking the
// lane quads {0,3,5,6}, {1,2,4,7}, {8,11,13,14} or {9,10,12,15} (quad j =
// lanes 4j..4j+3), and ds_write_b128 in eight passes of 8 consecutive lanes
// over 128 bytes.  With this f a fragment read (lane l: row R + l % 16 for R
// a multiple of 16, chunk l / 16) puts every read pass on 16 distinct 16-byte
// slots, the k-major loader (lane l: row R + l, one chunk) every write pass on
// 8, and the row loader (four lanes a row) writes whole rows: no bank
// conflicts.  Element offset of chunk c in row r:
__device__ __forceinline__ int swz(int r, int c) { return (c ^ ((r >> 1) & 3)) << 3; }

// Linear tile index -> (tm, tn); sym: the tiles with tm <= tn.
__device__ __forceinline__ void tile_of(int t, int tiles_n, bool sym, int& tm, int& tn) {
  if (!sym) {
    tm = t / tiles_n;
    tn = t - tm * tiles_n;
    return;
  }
  int row = 0;
  while (t >= tiles_n - row) { t -= tiles_n - row; ++row; }
  tm = row;
  tn = row + t;
}

// XM: X operand as planes (0), FP32 k-major X + b*sx + k*ldx + m (1), or FP32
// with rows contiguous X + b*sx + m*ldx + k, 16-byte aligned rows (2).
template <int XM, bool YPS, bool BIGK, int TS>
__device__ __forceinline__ void fx_body(const FxDesc& d, int tiles_n, int ntiles) {
  constexpr bool XPS = XM == 0;
  typedef Tile<TS> G;
  constexpr int FM = G::FM;
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][4][TS][KT];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][4][TS][KT];

  const int tid = threadIdx.x;
  const int l = tid & 63, w = tid >> 6;
  const int wm = w / G::WN, wn = w % G::WN;   // wave tile: rows WR*wm.., columns 32*wn..

  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  const int bb = logical / ntiles;
  int tm, tn;
  tile_of(logical - bb * ntiles, tiles_n, d.sym, tm, tn);
  long long ob = 0, ib = bb;                  // outer and inner batch index
  if (d.binner > 0) {
    ob = bb / d.binner;
    ib = bb - ob * d.binner;
  }
  const long long offx = ib * d.sx + ob * d.sx2, offy = ib * d.sy + ob * d.sy2;
  const int m0 = tm * TS, n0 = tn * TS;
  const int nstage = (d.K + KT - 1) / KT;

  // loaders: thread owns row cx of the X tile (column cy of Y) and its 8 k of
  // quarter kq.  Operands with k contiguous (planes, row-major X): the four
  // quarters of a row are neighbouring lanes, so one wave reads 16 rows of
  // 64-128 contiguous bytes; k-major FP32: lanes run along the row index.
  constexpr bool XKC = XM != 1;                 // X with k contiguous
  const int cx = XKC ? tid >> 2 : tid % TS, kqx = XKC ? tid & 3 : tid / TS;
  const int cy = YPS ? tid >> 2 : tid % TS, kqy = YPS ? tid & 3 : tid / TS;
  const bool xok = m0 + cx < d.M, yok = n0 + cy < d.N;
  const int ex = (!XPS && xok) ? d.ex[(long long)bb * d.sex + m0 + cx] : 0;
  const int ey = (!YPS && yok) ? d.ey[ib * d.sey + ob * d.sey2 + n0 + cy] : 0;

  // raw operands of one stage of this thread (planes as loaded, FP32 values
  // split when they are stored to LDS)
  struct Raw {
    bf8v xp[XPS ? 4 : 1], yp[YPS ? 4 : 1];
    float xr[XPS ? 1 : 8], yr[YPS ? 1 : 8];
  };

  auto load = [&](int s, Raw& R) {
    int k0 = s * KT + 8 * kqx;
    int kl = d.K - k0;
    if constexpr (XPS) {
      const __bf16* p = (const __bf16*)d.X + offx + (long long)(m0 + cx) * d.ldx + k0;
#pragma unroll
      for (int q = 0; q < 4; ++q) R.xp[XPS ? q : 0] = xok ? *(const bf8v*)(p + (long long)q * d.psx) : bf8v{};
    } else if constexpr (XM == 2) {
      const float* p = (const float*)d.X + offx + (long long)(m0 + cx) * d.ldx + k0;
      if (xok && kl >= 8) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const float4 f = *(const float4*)(p + 4 * v);
          R.xr[XPS ? 0 : 4 * v] = f.x; R.xr[XPS ? 0 : 4 * v + 1] = f.y;
          R.xr[XPS ? 0 : 4 * v + 2] = f.z; R.xr[XPS ? 0 : 4 * v + 3] = f.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) R.xr[XPS ? 0 : j] = (xok && j < kl) ? p[j] : 0.f;
      }
    } else {
      const float* p = (const float*)d.X + offx + (long long)k0 * d.ldx + m0 + cx;
#pragma unroll
      for (int j = 0; j < 8; ++j) R.xr[XPS ? 0 : j] = (xok && j < kl) ? p[(long long)j * d.ldx] : 0.f;
    }
    k0 = s * KT + 8 * kqy;
    kl = d.K - k0;
    if constexpr (YPS) {
      const __bf16* p = (const __bf16*)d.Y + offy + (long long)(n0 + cy) * d.ldy + k0;
#pragma unroll
      for (int q = 0; q < 4; ++q) R.yp[YPS ? q : 0] = yok ? *(const bf8v*)(p + (long long)q * d.psy) : bf8v{};
    } else {
      const float* p = (const float*)d.Y + offy + (long long)k0 * d.ldy + n0 + cy;
#pragma unroll
      for (int j = 0; j < 8; ++j) R.yr[YPS ? 0 : j] = (yok && j < kl) ? p[(long long)j * d.ldy] : 0.f;
    }
  };

  auto store = [&](const Raw& R, int buf) {
    if constexpr (XPS) {
#pragma unroll
      for (int q = 0; q < 4; ++q) *(bf8v*)&Xs[buf][q][cx][swz(cx, kqx)] = R.xp[XPS ? q : 0];
    } else {
      bf8v pk[4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        bf2v p[4];
        split_g2(f2v{R.xr[XPS ? 0 : e], R.xr[XPS ? 0 : e + 1]}, ex, p);
#pragma unroll
        for (int q = 0; q < 4; ++q) { pk[q][e] = p[q][0]; pk[q][e + 1] = p[q][1]; }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) *(bf8v*)&Xs[buf][q][cx][swz(cx, kqx)] = pk[q];
    }
    if constexpr (YPS) {
#pragma unroll
      for (int q = 0; q < 4; ++q) *(bf8v*)&Ys[buf][q][cy][swz(cy, kqy)] = R.yp[YPS ? q : 0];
    } else {
      bf8v pk[4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        bf2v p[4];
        split_g2(f2v{R.yr[YPS ? 0 : e], R.yr[YPS ? 0 : e + 1]}, ey, p);
#pragma unroll
        for (int q = 0; q < 4; ++q) { pk[q][e] = p[q][0]; pk[q][e + 1] = p[q][1]; }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) *(bf8v*)&Ys[buf][q][cy][swz(cy, kqy)] = pk[q];
    }
  };

  f4v acc0[FM][2], acc1[FM][2];
  d4v acc64[BIGK ? FM : 1][BIGK ? 2 : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc0[i][j] = f4v{0, 0, 0, 0};
      acc1[i][j] = f4v{0, 0, 0, 0};
      if (BIGK) acc64[BIGK ? i : 0][BIGK ? j : 0] = d4v{0, 0, 0, 0};
    }

  // fragment rows start at multiples of 16, so the swizzle of row l%16 applies
  const int kl = swz(l & 15, l >> 4);
  auto compute = [&](int s, int buf) {
    bf8v b[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) b[j][q] = *(const bf8v*)&Ys[buf][q][wn * 32 + j * 16 + (l & 15)][kl];
    // two row fragments at a time (four independent accumulators per step):
    // orders 3, 2, 1 into acc1 (smallest first), then the exact order 0
#pragma unroll
    for (int ip = 0; ip < FM; ip += 2) {
      bf8v a[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) a[i][q] = *(const bf8v*)&Xs[buf][q][wm * G::WR + (ip + i) * 16 + (l & 15)][kl];
#pragma unroll
      for (int o = 3; o >= 1; --o)
#pragma unroll
        for (int px = 0; px <= o; ++px) {
          const int py = o - px;
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc1[ip + i][j] =
                  __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][px], b[j][py], acc1[ip + i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc0[ip + i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], acc0[ip + i][j], 0, 0, 0);
    }
    if (BIGK && ((s + 1) % (EXACT_K / KT) == 0)) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[BIGK ? i : 0][BIGK ? j : 0][r] += (double)acc0[i][j][r];
          acc0[i][j] = f4v{0, 0, 0, 0};
        }
    }
  };

  // two LDS buffers, one barrier per stage.  Without the FP64 flush (K <=
  // 1024) two stages are in flight in registers: while stage s is multiplied
  // out of one buffer, stage s + 1 (loaded a stage earlier) is stored into
  // the other and stage s + 2 is being loaded; loads past the last stage
  // repeat it (in bounds) and go to a buffer nobody reads.  The flushing
  // variant has no registers to spare for that and keeps one stage in flight.
  if constexpr (!BIGK) {
    const int last = nstage - 1;
    Raw r0, r1;
    if (nstage > 0) {
      load(0, r0);
      load(min(1, last), r1);
      store(r0, 0);
    }
    __syncthreads();
    int s = 0;
    for (; s + 2 <= nstage; s += 2) {
      load(min(s + 2, last), r0);
      compute(s, 0);
      store(r1, 1);
      __syncthreads();
      load(min(s + 3, last), r1);
      compute(s + 1, 1);
      store(r0, 0);
      __syncthreads();
    }
    if (s < nstage) compute(s, 0);
  } else {
    Raw r0;
    if (nstage > 0) {
      load(0, r0);
      store(r0, 0);
    }
    __syncthreads();
    for (int s = 0; s < nstage; ++s) {
      const int buf = s & 1;
      if (s + 1 < nstage) load(s + 1, r0);
      compute(s, buf);
      if (s + 1 < nstage) store(r0, buf ^ 1);
      __syncthreads();
    }
  }

  float* __restrict__ Out = d.Out + ib * d.so + ob * d.so2;
  // bits of the largest |stored value| per column fragment, over the rows of
  // the tile's first slab (cm) and, with folded slabs, of the next (cm2:
  // rows from bnd on)
  int cm[2] = {0, 0}, cm2[2] = {0, 0};
  const int bnd = d.mslab > 0 ? (m0 / d.mslab + 1) * d.mslab : 0x7fffffff;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * G::WR + i * 16 + 4 * (l >> 4) + r;
        const int gn = n0 + wn * 32 + j * 16 + (l & 15);
        double v = (double)acc0[i][j][r] + (double)acc1[i][j][r];
        if (BIGK) v += acc64[BIGK ? i : 0][BIGK ? j : 0][r];
        if (gm >= d.M || gn >= d.N) continue;
        const float fv = (float)v;
        const int vb = (int)(__float_as_uint(fv) & 0x7fffffffu);
        if (gm < bnd)
          cm[j] = max(cm[j], vb);
        else
          cm2[j] = max(cm2[j], vb);
        if (!d.sym) {
          Out[(long long)gm * d.ldo + gn] = fv;
        } else if (gm <= gn) {
          Out[(long long)gm * d.ldo + gn] = fv;
          Out[(long long)gn * d.ldo + gm] = fv;
          if (gm == gn && d.Dg) d.Dg[ib * d.sd + ob * d.sd2 + gm] = v;
        }
      }
  if (d.cmax) {
    // column maxima of this tile's stored values (its rows only): over the
    // lane's rows, the four lane groups of a column, then the two row waves
    __shared__ int cms[2][2][TS];       // [slab part][wave row][column]
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cm[j] = max(cm[j], __shfl_xor(cm[j], 16, 64));
      cm[j] = max(cm[j], __shfl_xor(cm[j], 32, 64));
      cm2[j] = max(cm2[j], __shfl_xor(cm2[j], 16, 64));
      cm2[j] = max(cm2[j], __shfl_xor(cm2[j], 32, 64));
      if (l < 16) {
        cms[0][wm][wn * 32 + j * 16 + l] = cm[j];
        cms[1][wm][wn * 32 + j * 16 + l] = cm2[j];
      }
    }
    __syncthreads();
    if (tid < TS && n0 + tid < d.N) {
      const unsigned m1 = (unsigned)max(cms[0][0][tid], cms[0][1][tid]);
      if (d.mslab > 0) {
        d.cmax[(long long)tm * d.N + n0 + tid] = m1;
        if (min(m0 + TS, d.M) > bnd)      // the tile reaches into slab bnd / mslab
          d.cmax[d.scm + (long long)(bnd / d.mslab) * d.N + n0 + tid] =
              (unsigned)max(cms[1][0][tid], cms[1][1][tid]);
      } else {
        d.cmax[(long long)bb * d.scm + (long long)tm * d.N + n0 + tid] = m1;
      }
    }
  }
}

// Exchange-type generalized-Fock term of the split forms, on the tiling of
// the transform above:
//   Out_g[r][s] = sum_{P in group g} sum_q b^P[q][r] (S[q][s] b^P[q][s])
// b^P is symmetric, so both operands are read along rows (q contiguous); St
// is S transposed in FP32 (St[s][q]).  Each FP32 operand value is split into
// three BF16 pieces (x = hi + mid + lo exactly) and the six products of order
// <= 2 are accumulated in FP32 over two stages (64 q of one auxiliary slab),
// then added to FP64.
// The term enters lambda and the orbital gradient, not the energy.
// Three BF16 pieces of each of two values, x = hi + mid + lo exactly (each
// residual is exact in FP32): each BF16 rounding of a pair is one packed
// conversion, and the pieces come out packed as they are stored.
__device__ __forceinline__ void split3x2(f2v v, bf2v (&p)[3]) {
  p[0] = __builtin_convertvector(v, bf2v);
  const f2v r1 = v - __builtin_convertvector(p[0], f2v);
  p[1] = __builtin_convertvector(r1, bf2v);
  p[2] = __builtin_convertvector(r1 - __builtin_convertvector(p[1], f2v), bf2v);
}

// Raw operands of one stage of a lane: eight consecutive q of its X row, Y
// row and St row, loaded as they are; the masks, the S scaling and the split
// are applied when they are stored to LDS, so no instruction consumes a load
// in the stage that issues it (the wait for it falls after that stage's
// products).
struct ExRaw {
  float x[8], y[8], s[8];
};

// VEC: norb % 4 == 0 (rows 16-byte aligned): two float4 per row and stage, at
// addresses clamped into the row (a column block past the end re-reads the
// last four values, masked at the store).
template <bool VEC, int TS>
__device__ __forceinline__ void exch_body(const ExDesc& d, int tiles_n, int ntiles) {
  typedef Tile<TS> G;
  constexpr int FM = G::FM;
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][3][TS][KT];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][3][TS][KT];

  const int tid = threadIdx.x;
  const int l = tid & 63, w = tid >> 6;
  const int wm = w / G::WN, wn = w % G::WN;

  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  const int ngrp = (d.naux + d.fold - 1) / d.fold;
  const int inst = logical / (ngrp * ntiles);
  const int r = logical - inst * (ngrp * ntiles);
  const int grp = r / ntiles;
  const int t = r - grp * ntiles;
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int m0 = tm * TS, n0 = tn * TS;
  const int n = d.norb;
  const float* __restrict__ bI = d.b + (long long)inst * d.sb;
  const float* __restrict__ StI = d.St + (long long)inst * n * n;
  const int nkb = ((n + KT - 1) / KT + 1) & ~1;    // q-blocks, padded to pairs
  const int p_lo = grp * d.fold;
  const int p_hi = min(d.naux, p_lo + d.fold);
  const int np = p_hi - p_lo;
  const int nstage = np * nkb;

  const int c = tid >> 2, kq = tid & 3;       // row c of both tiles, k quarter kq
  const bool xok = m0 + c < n, yok = n0 + c < n;
  const int xrow = min(m0 + c, n - 1), yrow = min(n0 + c, n - 1);

  // Stages run in pairs over two consecutive q-blocks of one slab; the slabs
  // of the group run inside each pair of q-blocks: stage s covers q-block
  // 2 (s / 2np) + s % 2 of slab p_lo + (s / 2) % np.  The lane's St values
  // of a q-block are loaded once (on the first slab) and kept in sv while
  // the slabs pass; a q-block past the row end is all zeros (masked).
  auto qbase = [&](int s) { return (2 * (s / (2 * np)) + (s & 1)) * KT + 8 * kq; };
  auto load = [&](int s, ExRaw& r) {
    const int pb = p_lo + (s >> 1) % np;
    const bool first = (s >> 1) % np == 0;
    const int k0 = qbase(s);
    const float* bp = bI + (long long)pb * n * n;
    const float* px = bp + (long long)xrow * n;
    const float* py = bp + (long long)yrow * n;
    const float* ps = StI + (long long)yrow * n;
    if constexpr (VEC) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int k = min(k0 + 4 * v, n - 4);
        const float4 fx = *(const float4*)(px + k);
        const float4 fy = *(const float4*)(py + k);
        r.x[4 * v] = fx.x; r.x[4 * v + 1] = fx.y; r.x[4 * v + 2] = fx.z; r.x[4 * v + 3] = fx.w;
        r.y[4 * v] = fy.x; r.y[4 * v + 1] = fy.y; r.y[4 * v + 2] = fy.z; r.y[4 * v + 3] = fy.w;
        if (first) {
          const float4 fs = *(const float4*)(ps + k);
          r.s[4 * v] = fs.x; r.s[4 * v + 1] = fs.y; r.s[4 * v + 2] = fs.z; r.s[4 * v + 3] = fs.w;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = min(k0 + j, n - 1);
        r.x[j] = px[k];
        r.y[j] = py[k];
        if (first) r.s[j] = ps[k];
      }
    }
  };
  // sv[j]: St values of the q-block of the stages stored into LDS buffer j
  // (stage s goes to buffer s % 2; the clamped repeat of the last stage at
  // the end goes to a buffer nobody reads)
  float sv[2][8];
  auto store = [&](int s, const ExRaw& r, int buf) {
    const int kl = n - qbase(s);
    if ((s >> 1) % np == 0) {
#pragma unroll
      for (int e = 0; e < 8; ++e) sv[buf][e] = r.s[e];
    }
    // masks only where the tile or the row ends
    const bool full = kl >= 8;
    const bool xm = xok, ym = yok;
    bf8v px[3], py[3];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      f2v xv = {r.x[e], r.x[e + 1]};
      f2v yv = {r.y[e] * sv[buf][e], r.y[e + 1] * sv[buf][e + 1]};
      if (!(full && xm && ym)) {
        xv = f2v{(xm && e < kl) ? xv[0] : 0.f, (xm && e + 1 < kl) ? xv[1] : 0.f};
        yv = f2v{(ym && e < kl) ? yv[0] : 0.f, (ym && e + 1 < kl) ? yv[1] : 0.f};
      }
      bf2v a[3], b[3];
      split3x2(xv, a);
      split3x2(yv, b);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        px[q][e] = a[q][0]; px[q][e + 1] = a[q][1];
        py[q][e] = b[q][0]; py[q][e + 1] = b[q][1];
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      *(bf8v*)&Xs[buf][q][c][swz(c, kq)] = px[q];
      *(bf8v*)&Ys[buf][q][c][swz(c, kq)] = py[q];
    }
  };

  f4v acc[FM][2];
  d4v acc64[FM][2];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = f4v{0, 0, 0, 0};
      acc64[i][j] = d4v{0, 0, 0, 0};
    }

  const int kl = swz(l & 15, l >> 4);
  auto compute = [&](int s, int buf) {
    bf8v b[2][3];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 3; ++q) b[j][q] = *(const bf8v*)&Ys[buf][q][wn * 32 + j * 16 + (l & 15)][kl];
#pragma unroll
    for (int ip = 0; ip < FM; ip += 2) {
      bf8v a[2][3];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) a[i][q] = *(const bf8v*)&Xs[buf][q][wm * G::WR + (ip + i) * 16 + (l & 15)][kl];
#pragma unroll
      for (int o = 2; o >= 0; --o)
#pragma unroll
        for (int px = 0; px <= o; ++px) {
          const int py = o - px;
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[ip + i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][px], b[j][py], acc[ip + i][j], 0, 0, 0);
        }
    }
    if (s & 1) {   // each pair's FP32 sums (64 q of one slab) into FP64: the
                   // result does not depend on how the slabs are grouped
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = f4v{0, 0, 0, 0};
        }
    }
  };

  // two stages in flight in registers: at stage s the registers of s (stored
  // to LDS already) are refilled with stage s + 2, clamped to the last stage
  // (the final loads repeat it and are stored to a buffer nobody reads)
  const int last = nstage - 1;
  ExRaw r0, r1;
  if (nstage > 0) {
    load(0, r0);
    load(min(1, last), r1);
    store(0, r0, 0);
  }
  __syncthreads();
  int s = 0;
  for (; s + 2 <= nstage; s += 2) {
    load(min(s + 2, last), r0);
    compute(s, 0);
    store(s + 1, r1, 1);
    __syncthreads();
    load(min(s + 3, last), r1);
    compute(s + 1, 1);
    store(min(s + 2, last), r0, 0);
    __syncthreads();
  }
  if (s < nstage) compute(s, 0);

  double* __restrict__ Out = d.Out + (long long)inst * d.so + (long long)grp * n * n;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * G::WR + i * 16 + 4 * (l >> 4) + r;
        const int gn = n0 + wn * 32 + j * 16 + (l & 15);
        if (gm < n && gn < n) Out[(long long)gm * n + gn] = acc64[i][j][r];
      }
}

template <bool VEC, int TS>
__global__ __launch_bounds__(Tile<TS>::NT, Tile<TS>::MINB) void k_exchange_fock_fx(ExDesc d, int tiles_n,
                                                                                    int ntiles) {
  exch_body<VEC, TS>(d, tiles_n, ntiles);
}

// St_i[s][q] = (float)S_i[q][s] for ninst matrices n^2 apart
__global__ void k_transpose_f32(const double* __restrict__ S, int n, int ninst, float* __restrict__ St) {
  const long long nn = (long long)n * n, total = nn * ninst;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long y = i / nn, e = i - y * nn;
    const long long s = e / n, q = e - s * n;
    St[i] = (float)S[y * nn + q * n + s];
  }
}

#define NOF_FX_KERNEL(NAME)                                                               \
  template <int XM, bool YPS, bool BIGK, int TS>                                          \
  __global__ __launch_bounds__(Tile<TS>::NT, Tile<TS>::MINB) void NAME(FxDesc d, int tiles_n, \
                                                                       int ntiles) {      \
    fx_body<XM, YPS, BIGK, TS>(d, tiles_n, ntiles);                                       \
  }
NOF_FX_KERNEL(k_transform_stage1_fx)
NOF_FX_KERNEL(k_transform_stage2_fx)
#undef NOF_FX_KERNEL

template <int XM, bool YPS, bool BIGK, int TS = 128>
int launch_fx(const FxDesc& d, hipStream_t st) {
  const int tiles_m = (d.M + TS - 1) / TS;
  const int tiles_n = (d.N + TS - 1) / TS;
  const int ntiles = d.sym ? tiles_n * (tiles_n + 1) / 2 : tiles_m * tiles_n;
  const long long G = (long long)ntiles * d.batch;
  if (G <= 0) return NOF_OK;
  if (G > 0x7fffffffLL) return NOF_E_DIM;
  if (d.role == 1)
    hipLaunchKernelGGL((k_transform_stage1_fx<XM, YPS, BIGK, TS>), dim3((unsigned)G), dim3(Tile<TS>::NT), 0,
                       st, d, tiles_n, ntiles);
  else
    hipLaunchKernelGGL((k_transform_stage2_fx<XM, YPS, BIGK, TS>), dim3((unsigned)G), dim3(Tile<TS>::NT), 0,
                       st, d, tiles_n, ntiles);
  return launch_status();
}

long long grid_for(long long items, int per_block) {
  long long g = (items + per_block - 1) / per_block;
  return g < 1 ? 1 : (g > 65536 ? 65536 : g);
}

template <int TS>
int launch_exchange_fx(const ExDesc& d, hipStream_t st) {
  const int tiles_n = (d.norb + TS - 1) / TS;
  const int ntiles = tiles_n * tiles_n;
  const int groups = (d.naux + d.fold - 1) / d.fold;
  const long long G = (long long)ntiles * groups * d.ninst;
  if (G > 0x7fffffffLL) return NOF_E_DIM;
  if (d.norb % 4 == 0)
    hipLaunchKernelGGL((k_exchange_fock_fx<true, TS>), dim3((unsigned)G), dim3(Tile<TS>::NT), 0, st, d, tiles_n,
                       ntiles);
  else
    hipLaunchKernelGGL((k_exchange_fock_fx<false, TS>), dim3((unsigned)G), dim3(Tile<TS>::NT), 0, st, d,
                       tiles_n, ntiles);
  return launch_status();
}

}  // namespace

int gemm_fx(const FxDesc& d, bool x_planes, bool y_planes, hipStream_t st) {
  if (d.M < 0 || d.N < 0 || d.K < 0 || d.batch < 0) return NOF_E_DIM;
  if (d.sym && (d.M != d.N)) return NOF_E_DIM;
  if ((!x_planes && !d.ex) || (!y_planes && !d.ey)) return NOF_E_NULL;
  if (d.binner < 0 || (d.binner > 0 && (d.cmax || d.batch % d.binner))) return NOF_E_ARG;
  if (d.tile != 128 && d.tile != 64) return NOF_E_ARG;
  if (d.mslab < 0) return NOF_E_ARG;
  // folded slabs: X as planes (rows (P, mu) contiguous), one batch entry
  if (d.mslab > 0 && (!x_planes || d.batch != 1 || d.sym || d.binner || d.mslab < d.tile || d.M % d.mslab ||
                      (long long)d.M + d.mslab > 0x7fffffffLL))
    return NOF_E_ARG;
  const bool big = d.K > EXACT_K;
  // 64-wide tiles for pre-split X only (the batched transform stages)
  if (d.tile == 64) {
    if (!x_planes) return NOF_E_ARG;
    if (y_planes)
      return big ? launch_fx<0, true, true, 64>(d, st) : launch_fx<0, true, false, 64>(d, st);
    return big ? launch_fx<0, false, true, 64>(d, st) : launch_fx<0, false, false, 64>(d, st);
  }
  if (x_planes && y_planes)
    return big ? launch_fx<0, true, true>(d, st) : launch_fx<0, true, false>(d, st);
  if (x_planes && !y_planes)
    return big ? launch_fx<0, false, true>(d, st) : launch_fx<0, false, false>(d, st);
  if (!y_planes) return NOF_E_DTYPE;
  if (d.x_rows) {
    // rows contiguous: float4 loads when every row start is 16-byte aligned
    if (d.ldx % 4 == 0 && d.sx % 4 == 0 && ((uintptr_t)d.X & 15) == 0)
      return big ? launch_fx<2, true, true>(d, st) : launch_fx<2, true, false>(d, st);
    // otherwise the same values read k-major (the operand is symmetric)
  }
  return big ? launch_fx<1, true, true>(d, st) : launch_fx<1, true, false>(d, st);
}

int fx_transpose(const double* S, int n, int ninst, float* St, hipStream_t st) {
  if (n <= 0 || ninst <= 0) return NOF_E_DIM;
  const long long nn = (long long)n * n;
  hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)grid_for(nn * ninst, 256)), dim3(256), 0, st, S, n, ninst,
                     St);
  return launch_status();
}

int exchange_fock_fx(const ExDesc& d0, const double* S, float* St, hipStream_t st) {
  if (d0.naux <= 0 || d0.norb <= 0 || d0.fold <= 0 || d0.ninst <= 0) return NOF_E_DIM;
  if (d0.tile != 128 && d0.tile != 64) return NOF_E_ARG;
  const long long nn = (long long)d0.norb * d0.norb;
  hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)grid_for(nn * d0.ninst, 256)), dim3(256), 0, st, S,
                     d0.norb, d0.ninst, St);
  const int rc = launch_status();
  if (rc != NOF_OK) return rc;
  ExDesc d = d0;
  d.St = St;
  return d.tile == 64 ? launch_exchange_fx<64>(d, st) : launch_exchange_fx<128>(d, st);
}

int fx_row_exps(const void* A, int At, long long nrow, int K, int* e, hipStream_t st) {
  if (nrow <= 0 || K <= 0) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_for(nrow, 4);
  if (At == NOF_F64)
    hipLaunchKernelGGL(k_row_exps<double>, dim3(g), dim3(256), 0, st, (const double*)A, nrow, K, e);
  else if (At == NOF_F32)
    hipLaunchKernelGGL(k_row_exps<float>, dim3(g), dim3(256), 0, st, (const float*)A, nrow, K, e);
  else
    return NOF_E_DTYPE;
  return launch_status();
}

int fx_col_exps(const float* A, int batch, int K, int N, long long sa, int* e, hipStream_t st) {
  if (batch <= 0 || K <= 0 || N <= 0) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_for((long long)batch * ((N + 63) / 64), 1);
  hipLaunchKernelGGL(k_col_exps, dim3(g), dim3(256), 0, st, A, batch, K, N, sa, e);
  return launch_status();
}

int fx_cmax_exps(const unsigned* cmax, int batch, int tiles, int N, int* e, hipStream_t st, int mslab,
                 int ts) {
  if (batch <= 0 || tiles <= 0 || N <= 0 || mslab < 0 || (mslab > 0 && (ts <= 0 || mslab < ts)))
    return NOF_E_DIM;
  const unsigned g = (unsigned)grid_for((long long)batch * N, 256);
  hipLaunchKernelGGL(k_cmax_exps, dim3(g), dim3(256), 0, st, cmax, (long long)batch, tiles, N, e, mslab, ts);
  return launch_status();
}

int fx_split_cols(const double* A, int K, int ncol, int lda, int ldk, void* out, hipStream_t st) {
  if (K <= 0 || ncol <= 0 || ldk < K || ldk % KT) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_for(ncol, 16);
  hipLaunchKernelGGL(k_split_cols, dim3(g), dim3(256), 0, st, A, K, ncol, lda, ldk, (__bf16*)out);
  return launch_status();
}

int fx_split_rows(const void* A, int At, long long nrow, int K, int ldk, void* out, hipStream_t st) {
  if (nrow <= 0 || K <= 0 || ldk < K || ldk % KT) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_for(nrow, 4);
  if (At == NOF_F64)
    hipLaunchKernelGGL(k_split_rows<double>, dim3(g), dim3(256), 0, st, (const double*)A, nrow, K, ldk,
                       (__bf16*)out);
  else if (At == NOF_F32)
    hipLaunchKernelGGL(k_split_rows<float>, dim3(g), dim3(256), 0, st, (const float*)A, nrow, K, ldk,
                       (__bf16*)out);
  else
    return NOF_E_DTYPE;
  return launch_status();
}

}  // namespace nof
