// INT8 form of the fixed-point split transform (NOF_P_I8X10): the two
// stages of the orbital transformation, b^P = C^T B^P C, on the INT8 matrix
// cores.
//
//   Out_b[m][n] = sum_k X_b(k, m) * Y_b(k, n)
//
// As in the BF16 fixed-point form, every row m of X and every column n of Y
// gets one grid over the whole contraction (Ozaki, Ogita, Oishi and Rump,
// Numer. Algorithms 2012: error-free splitting against a per-vector grid), here
// with INT8 pieces: with 2^E the smallest power of two for which
// max|x| 2^(7-E) < 127.5,
//   x = n_0 2^(E-7) + n_1 2^(E-14) + n_2 2^(E-21) + n_3 2^(E-28) + r,
//   |n_0| <= 127, |n_1|, |n_2|, |n_3| <= 64, |r| <= 2^(E-29)
// (each piece rounds what the previous ones left, at most half a unit of
// their grid, on a grid 2^7 finer).  A product of pieces of order
// o = qx + qy counts units of 2^(Ex+Ey-14-7o); v_mfma_i32_16x16x64_i8 sums 64
// of them per instruction exactly in int32, and the ten products of order
// <= 3 go to four accumulators, one per order.  Per k an order adds at most
// 2*127*64 + 2*64^2 = 24448 units, so the sums are exact for K < 87,000.  The
// epilogue forms
//   v = 2^(Ex+Ey-14) (acc0 + 2^-7 (acc1 + 2^-7 (acc2 + 2^-7 acc3)))
// in FP64, where every step is exact (at most 52 significant bits).  What
// remains is the representation residual r (2^-29 of a vector's largest
// element) and the dropped products of order 4..6 (below 2^-28 of
// |x|max |y|max per term).
//
// Against the BF16 form: the pieces are half the bytes, an instruction does
// twice the multiply-adds at the same issue rate, and the accumulators never
// round, so no FP64 flush is needed at any depth.
//
// Operands are planes [4][rows][ldk] of INT8 (k contiguous, ldk a multiple
// of 64, zero past K) with one int32 grid exponent per row.
//
// Layout: 512 threads = 8 waves (2 x 4); the workgroup tile is 128 x 128,
// each wave 64 x 32 as 4 x 2 fragments of v_mfma_i32_16x16x64_i8 (lane l
// holds 16 consecutive k of row l%16 at k offset 16*(l/16), the same 16-byte
// operand layout as the BF16 16x16x32 instruction; output row 4*(l/16)+r,
// column l%16).  LDS holds the four planes as [row][64 k] (16-byte chunks
// swizzled by row), double-buffered; the next stage's loads are in flight
// while the current one is multiplied.
#include "common.h"

namespace nof {
namespace {

typedef int i4v __attribute__((ext_vector_type(4)));

constexpr int IT = 128;                 // tile edge
constexpr int IK = 64;                  // k per stage (bytes per LDS row)
constexpr int INTHR = 512;
constexpr int IEMIN = -90, IEMAX = 128; // grid exponent range (FP32 scales stay normal)

__device__ __forceinline__ int xcd_logical(int w, int G) {
  const int q = G >> 3, r = G & 7, x = w & 7, i = w >> 3;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int clamp_e(int e) { return e < IEMIN ? IEMIN : (e > IEMAX ? IEMAX : e); }

// Grid exponent of a vector whose largest magnitude is m (FP64).
__device__ __forceinline__ int grid_exp_i8(double m) {
  if (!(m > 0.0)) return IEMIN;
  int E;
  frexp(m, &E);                          // m < 2^E
  if (ldexp(m, 7 - E) >= 127.5) ++E;
  return clamp_e(E);
}

// The same from the bits of a non-negative FP32 maximum.
__device__ __forceinline__ int grid_exp_i8_bits(unsigned mbits) {
  if (mbits == 0) return IEMIN;
  int E = (int)(mbits >> 23) - 126;      // 2^E > m, m 2^(7-E) in [64, 128)
  if ((mbits & 0x7fffffu) >= 0x7f0000u) ++E;   // m 2^(7-E) >= 127.5
  return clamp_e(E);
}

// Pieces of v on the grid of exponent E, packed: byte q of the result is n_q.
__device__ __forceinline__ void split_i8(double v, int E, unsigned (&p)[4], int byte) {
  double t = ldexp(v, 7 - E);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double n = rint(t);
    p[q] |= ((unsigned)(int)n & 0xffu) << (8 * byte);
    t = (t - n) * 128.0;
  }
}

// The same for an FP32 value, each rounding done by adding 1.5 * 2^23: for
// |t| < 2^22 the sum lies in [2^23, 2^24), where the FP32 spacing is 1, so it
// is M + rint(t) (ties to even, as rintf) and its low mantissa byte is
// rint(t) mod 256, the piece's byte, with no conversion to integer.
__device__ __forceinline__ void split_i8f(float v, int E, unsigned (&p)[4], int byte) {
  constexpr float M = 12582912.0f;       // 1.5 * 2^23
  float t = v * __int_as_float((127 + 7 - E) << 23);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float u = t + M;
    p[q] |= (__float_as_uint(u) & 0xffu) << (8 * byte);
    if (q < 3) t = (t - (u - M)) * 128.0f;
  }
}

// Planes and grid exponents of the rows of A[nrow][K] (FP64 or FP32, rows
// contiguous): out[q][row][ldk], e[row]; one wave per row, lane l splits
// four consecutive k per step (one 32-bit store per plane).
template <typename T>
__global__ void k_split_rows_i8(const T* __restrict__ A, long long nrow, int K, int ldk,
                                unsigned char* __restrict__ out, int* __restrict__ e) {
  const int l = threadIdx.x & 63;
  const long long wpb = blockDim.x >> 6;
  const long long plane = nrow * ldk;
  for (long long row = blockIdx.x * wpb + (threadIdx.x >> 6); row < nrow; row += (long long)gridDim.x * wpb) {
    const T* a = A + row * K;
    double m = 0.0;
    for (int k = l; k < K; k += 64) m = fmax(m, fabs((double)a[k]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    const int E = grid_exp_i8(m);
    if (l == 0) e[row] = E;
    for (int k4 = 4 * l; k4 < ldk; k4 += 256) {
      unsigned p[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int i = 0; i < 4; ++i) split_i8(k4 + i < K ? (double)a[k4 + i] : 0.0, E, p, i);
#pragma unroll
      for (int q = 0; q < 4; ++q) *(unsigned*)(out + q * plane + row * ldk + k4) = p[q];
    }
  }
}

// Planes and grid exponents of the columns of an FP64 k-major A[k][col]
// (k < K): out[q][col][ldk], e[col].  Block: 16 columns; their maxima from 16
// row groups, then each wave splits four columns with lanes along k.
__global__ void k_split_cols_i8(const double* __restrict__ A, int K, int ncol, int lda, int ldk,
                                unsigned char* __restrict__ out, int* __restrict__ e) {
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
      ecol[c] = grid_exp_i8(mm);
      if (c0 + c < ncol) e[c0 + c] = ecol[c];
    }
    __syncthreads();
    for (int cc = 4 * w; cc < 4 * w + 4; ++cc) {
      const int col = c0 + cc;
      if (col >= ncol) break;
      for (int k4 = 4 * l; k4 < ldk; k4 += 256) {
        unsigned p[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < 4; ++i)
          split_i8(k4 + i < K ? A[(long long)(k4 + i) * lda + col] : 0.0, ecol[cc], p, i);
#pragma unroll
        for (int q = 0; q < 4; ++q) *(unsigned*)(out + q * plane + (long long)col * ldk + k4) = p[q];
      }
    }
    __syncthreads();
  }
}

// Grid exponents of the columns of T_b (FP32) from the per-row-tile column
// maxima of the stage-1 epilogue: e[b*N + n] from max_t cmax[b][t][n], or
// (mslab > 0) from the folded layout (slab_cmax, tile edge IT).
__global__ void k_cmax_exps_i8(const unsigned* __restrict__ cmax, long long batch, int tiles, int N,
                               int* __restrict__ e, int mslab) {
  const long long total = batch * N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long b = i / N;
    const int n = (int)(i - b * N);
    unsigned m = 0;
    if (mslab > 0) {
      m = slab_cmax(cmax, b, mslab, IT, tiles, N, n);
    } else {
      const unsigned* c = cmax + b * tiles * N + n;
      for (int t = 0; t < tiles; ++t) m = max(m, c[(long long)t * N]);
    }
    e[i] = grid_exp_i8_bits(m);
  }
}

// Planes of the columns of the k-major FP32 T_b[K][N] (batch stride sT, row
// stride ldt) on the grids e[b*N + n]: out[q][b][n][ldk].  Block: 64 columns x 128 k.  The
// split runs with lanes along n (coalesced reads of T's rows), 32 k per
// thread, into an LDS tile [q][n][k]; the tile is then written with lanes
// along k, so a wave stores eight whole 128-byte rows.
constexpr int TS_N = 64, TS_K = 128, TS_ROW = TS_K + 16;   // LDS row: 144 bytes (no conflicts)
__global__ void k_split_T_i8(const float* __restrict__ T, long long batch, int K, int N, long long sT,
                             long long ldt, int ldk, const int* __restrict__ e, unsigned char* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) unsigned char L[4][TS_N][TS_ROW];
  const int nkb = (ldk + TS_K - 1) / TS_K;
  const int ncb = (N + TS_N - 1) / TS_N;
  const long long blocks = batch * ncb * nkb;
  const long long plane = batch * (long long)N * ldk;
  const int t = threadIdx.x;
  const int nl = t & 63, kc = t >> 6;
  for (long long blk = blockIdx.x; blk < blocks; blk += gridDim.x) {
    const int kb = (int)(blk % nkb);
    const long long r = blk / nkb;
    const int cb = (int)(r % ncb);
    const long long b = r / ncb;
    const int n0 = cb * TS_N, k0 = kb * TS_K;
    // split: column n0 + nl, k = k0 + 32 kc .. + 32
    {
      const int n = min(n0 + nl, N - 1);
      const int E = e[b * N + n];
      const float* tp = T + b * sT + n;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        unsigned p[4][4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          unsigned pw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = k0 + 32 * kc + 16 * h + 4 * w + i;
            split_i8f(k < K ? tp[(long long)k * ldt] : 0.f, E, pw, i);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) p[q][w] = pw[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *(i4v*)&L[q][nl][32 * kc + 16 * h] = i4v{(int)p[q][0], (int)p[q][1], (int)p[q][2], (int)p[q][3]};
      }
    }
    __syncthreads();
    // store: chunk c of row (q, nr), 16 bytes; eight lanes per 128-byte row
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = t + 256 * j;
      const int c = idx & 7, nr = (idx >> 3) & 63, q = idx >> 9;
      const int k = k0 + 16 * c;
      if (n0 + nr < N && k < ldk)
        *(i4v*)(out + q * plane + (b * N + n0 + nr) * (long long)ldk + k) = *(const i4v*)&L[q][nr][16 * c];
    }
    __syncthreads();
  }
}

// Byte offset of 16-byte chunk c in LDS row r (64-byte rows): chunk c sits
// at position c ^ f(r), f(r) = (r / 2) mod 4.  On gfx950 ds_read_b128 serves a
// wave in four passes of 16 lanes over 256 bytes of banks, a pass taking the
// lane quads {0,3,5,6}, {1,2,4,7}, {8,11,13,14} or {9,10,12,15} (quad j =
// lanes 4j..4j+3; measured with the bank-conflict counter over lane-address
// patterns): with this f a fragment read (lane l: row R + l % 16 for R a
// multiple of 16, chunk l / 16) puts every pass on 16 distinct 16-byte
// slots.  The loader lanes (four per row) write whole 64-byte rows, which
// ds_write_b128 (eight passes of 8 consecutive lanes over 128 bytes) takes
// without conflicts.
__device__ __forceinline__ int swz16(int r, int c) { return (c ^ ((r >> 1) & 3)) << 4; }

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

__device__ __forceinline__ void i8_body(const I8Desc& d, int tiles_n, int ntiles) {
  __shared__ __attribute__((aligned(16))) unsigned char Xs[2][4][IT][IK];
  __shared__ __attribute__((aligned(16))) unsigned char Ys[2][4][IT][IK];

  const int tid = threadIdx.x;
  const int l = tid & 63, w = tid >> 6;
  const int wm = w >> 2, wn = w & 3;          // wave tile: rows 64*wm.., columns 32*wn..

  const int logical = xcd_logical(blockIdx.x, gridDim.x);
  const int bb = logical / ntiles;
  int tm, tn;
  tile_of(logical - bb * ntiles, tiles_n, d.sym, tm, tn);
  const int m0 = tm * IT, n0 = tn * IT;
  const int nstage = (d.K + IK - 1) / IK;
  long long ob = 0, ib = bb;                  // outer and inner batch index
  if (d.binner > 0) {
    ob = bb / d.binner;
    ib = bb - ob * d.binner;
  }

  // loader: thread owns row c of both tiles and the 16-byte chunk kq of it;
  // rows past the edge load the last row (in bounds, unconditional) and only
  // feed outputs that are never written
  const int c = tid >> 2, kq = tid & 3;
  const unsigned char* __restrict__ xrow =
      d.X + ib * d.sx + ob * d.sx2 + (long long)min(m0 + c, d.M - 1) * d.ldx + 16 * kq;
  const unsigned char* __restrict__ yrow =
      d.Y + ib * d.sy + ob * d.sy2 + (long long)min(n0 + c, d.N - 1) * d.ldy + 16 * kq;

  struct Raw {
    i4v x[4], y[4];
  };
  auto load = [&](int s, Raw& R) {
    const long long k0 = (long long)s * IK;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      R.x[q] = *(const i4v*)(xrow + q * d.psx + k0);
      R.y[q] = *(const i4v*)(yrow + q * d.psy + k0);
    }
  };
  auto store = [&](const Raw& R, int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *(i4v*)&Xs[buf][q][c][swz16(c, kq)] = R.x[q];
      *(i4v*)&Ys[buf][q][c][swz16(c, kq)] = R.y[q];
    }
  };

  i4v acc[4][4][2];                           // [order][row fragment][column fragment]
#pragma unroll
  for (int o = 0; o < 4; ++o)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[o][i][j] = i4v{0, 0, 0, 0};

  // fragment rows start at multiples of 16, so the swizzle of row l%16 applies
  const int kl = swz16(l & 15, l >> 4);
  auto compute = [&](int buf) {
    i4v b[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) b[j][q] = *(const i4v*)&Ys[buf][q][wn * 32 + j * 16 + (l & 15)][kl];
    // one piece of the row fragment at a time (piece px meets pieces
    // py <= 3 - px of the columns); consecutive instructions go to
    // different accumulators
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int px = 0; px < 4; ++px) {
        const i4v a = *(const i4v*)&Xs[buf][px][wm * 64 + i * 16 + (l & 15)][kl];
#pragma unroll
        for (int py = 0; py + px < 4; ++py)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[px + py][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b[j][py], acc[px + py][i][j], 0, 0, 0);
      }
  };

  // two LDS buffers, one barrier per stage; stage s + 1 is loaded while
  // stage s is multiplied and stored into the other buffer afterwards (a
  // second stage in flight does not fit beside the four accumulators)
  Raw r0;
  if (nstage > 0) {
    load(0, r0);
    store(r0, 0);
  }
  __syncthreads();
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    if (s + 1 < nstage) load(s + 1, r0);
    compute(buf);
    if (s + 1 < nstage) store(r0, buf ^ 1);
    __syncthreads();
  }

  float* __restrict__ Out = d.Out + ib * d.so + ob * d.so2;
  double* __restrict__ Dg = d.Dg ? d.Dg + ib * d.sd + ob * d.sd2 : nullptr;
  const int* __restrict__ ex = d.ex + ib * d.sex + ob * d.sex2;
  const int* __restrict__ ey = d.ey + ib * d.sey + ob * d.sey2;
  int eyc[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int gn = n0 + wn * 32 + j * 16 + (l & 15);
    eyc[j] = gn < d.N ? ey[gn] : 0;
  }
  // bits of the largest |stored value| per column fragment, over the rows of
  // the tile's first slab (cm) and, with folded slabs, of the next (cm2:
  // rows from bnd on)
  int cm[2] = {0, 0}, cm2[2] = {0, 0};
  const int bnd = d.mslab > 0 ? (m0 / d.mslab + 1) * d.mslab : 0x7fffffff;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wm * 64 + i * 16 + 4 * (l >> 4) + r;
      if (gm >= d.M) continue;
      const int exr = ex[gm];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gn = n0 + wn * 32 + j * 16 + (l & 15);
        if (gn >= d.N) continue;
        double v = (double)acc[3][i][j][r];
        v = (double)acc[2][i][j][r] + v * 0.0078125;
        v = (double)acc[1][i][j][r] + v * 0.0078125;
        v = (double)acc[0][i][j][r] + v * 0.0078125;
        v = ldexp(v, exr + eyc[j] - 14);
        if (d.Out64) {
          double* o = d.Out64 + ib * d.so + ob * d.so2;
          if (!d.sym) {
            o[(long long)gm * d.ldo + gn] = v;
          } else if (gm <= gn) {
            o[(long long)gm * d.ldo + gn] = v;
            o[(long long)gn * d.ldo + gm] = v;
          }
          continue;
        }
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
          if (gm == gn && Dg) Dg[gm] = v;
        }
      }
    }
  if (d.cmax) {
    // column maxima of this tile's stored values over its rows: the lane's
    // rows, the four lane groups of a column, then the two row waves
    __shared__ int cms[2][2][IT];       // [slab part][wave row][column]
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
    if (tid < IT && n0 + tid < d.N) {
      const unsigned m1 = (unsigned)max(cms[0][0][tid], cms[0][1][tid]);
      if (d.mslab > 0) {
        d.cmax[(long long)tm * d.N + n0 + tid] = m1;
        if (min(m0 + IT, d.M) > bnd)      // the tile reaches into slab bnd / mslab
          d.cmax[d.scm + (long long)(bnd / d.mslab) * d.N + n0 + tid] =
              (unsigned)max(cms[1][0][tid], cms[1][1][tid]);
      } else {
        d.cmax[bb * d.scm + (long long)tm * d.N + n0 + tid] = m1;
      }
    }
  }
}

__global__ __launch_bounds__(INTHR, 1) void k_transform_stage1_i8(I8Desc d, int tiles_n, int ntiles) {
  i8_body(d, tiles_n, ntiles);
}
__global__ __launch_bounds__(INTHR, 1) void k_transform_stage2_i8(I8Desc d, int tiles_n, int ntiles) {
  i8_body(d, tiles_n, ntiles);
}
__global__ __launch_bounds__(INTHR, 1) void k_exchange_fock_i8(I8Desc d, int tiles_n, int ntiles) {
  i8_body(d, tiles_n, ntiles);
}

// ---------------------------------------------------------------------------
// Exchange-type Fock term of the INT8 form.  The sum over the slabs of a group
// and over q is one contraction of length fold * ldk: row r of X^g holds
// b^P[r][q] slab after slab (each slab's segment padded to ldk with zeros), row
// s of Y^g holds St[s][q] b^P[s][q] (the FP32 product the split forms use), and
// each row of X^g and Y^g gets one grid over the whole group.
// ---------------------------------------------------------------------------

// Row maxima per slab: mx = max_q |b^P[s][q]|, my = max_q |St[s][q] b^P[s][q]|
// for every (instance, P, s); 16 lanes per row (four rows a wave), 16-byte
// loads when every row starts on a 16-byte boundary (V4: norb and sb
// multiples of 4).
template <bool V4>
__global__ void k_exch_rowmax_i8(const float* __restrict__ b, long long sb, const float* __restrict__ St,
                                 int ninst, int naux, int norb, float* __restrict__ mx,
                                 float* __restrict__ my) {
  const int l = threadIdx.x & 15;
  const long long rows = (long long)ninst * naux * norb;
  const long long rpb = blockDim.x >> 4;
  for (long long row0 = (long long)blockIdx.x * rpb; row0 < rows; row0 += (long long)gridDim.x * rpb) {
    const long long row = row0 + (threadIdx.x >> 4);
    const bool live = row < rows;                    // every lane reaches the shuffles
    const long long rr = live ? row : 0;
    const long long i = rr / ((long long)naux * norb);
    const long long ps = rr - i * naux * norb;        // P * norb + s
    const int s = (int)(ps % norb);
    const float* br = b + i * sb + ps * norb;
    const float* sr = St + (i * norb + s) * (long long)norb;
    float ax = 0.f, ay = 0.f;
    if (V4) {
      for (int q = 4 * l; live && q < norb; q += 64) {
        const float4 x = *(const float4*)(br + q), t = *(const float4*)(sr + q);
        ax = fmaxf(ax, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
        ay = fmaxf(ay, fmaxf(fmaxf(fabsf(t.x * x.x), fabsf(t.y * x.y)), fmaxf(fabsf(t.z * x.z), fabsf(t.w * x.w))));
      }
    } else {
      for (int q = l; live && q < norb; q += 16) {
        const float x = br[q];
        ax = fmaxf(ax, fabsf(x));
        ay = fmaxf(ay, fabsf(sr[q] * x));
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      ax = fmaxf(ax, __shfl_xor(ax, o, 64));
      ay = fmaxf(ay, __shfl_xor(ay, o, 64));
    }
    if (live && l == 0) {
      mx[row] = ax;
      my[row] = ay;
    }
  }
}

// Grid exponents per (instance, group, row) from the group's slab maxima.
__global__ void k_exch_grids_i8(const float* __restrict__ mx, const float* __restrict__ my, int ninst,
                                int naux, int norb, int fold, int ngroups, int* __restrict__ ex,
                                int* __restrict__ ey) {
  const long long total = (long long)ninst * ngroups * norb;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long i = t / ((long long)ngroups * norb);
    const long long gs = t - i * ngroups * norb;
    const int g = (int)(gs / norb), s = (int)(gs - (long long)g * norb);
    unsigned bx = 0, by = 0;
    const int p1 = min(naux, (g + 1) * fold);
    for (int P = g * fold; P < p1; ++P) {
      const long long r = (i * naux + P) * (long long)norb + s;
      bx = max(bx, __float_as_uint(mx[r]));
      by = max(by, __float_as_uint(my[r]));
    }
    ex[t] = grid_exp_i8_bits(bx);
    ey[t] = grid_exp_i8_bits(by);
  }
}

// Pieces of 16 consecutive values on the grid of exponent E: byte k of
// plane q is n_q of value k.
__device__ __forceinline__ void split16_i8(const float (&v)[16], int E, i4v (&p)[4]) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    unsigned u[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 4; ++k) split_i8f(v[4 * w + k], E, u, k);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q][w] = (int)u[q];
  }
}

// The planes: for every (instance, slab slot P < ngroups * fold, row s), the
// segment (P - g fold) * ldk .. + ldk of rows s of X^g and Y^g (zeros for
// q >= norb and for slots past the last slab).  Work item = one 16-byte
// chunk (16 consecutive q) of one such row, items in row order; a wave takes
// a contiguous range of items, lane l every 64th from its start, so short
// rows do not leave lanes idle, and a lane's (row, chunk) advances by
// additions (the divisions are done once).  One 16-byte store per plane; the
// values are loaded as four 16-byte vectors when V4 (rows of b and St
// 16-byte aligned) and the chunk lies inside the row.
template <bool V4>
__global__ void k_exch_split_i8(const float* __restrict__ b, long long sb, const float* __restrict__ St,
                                int ninst, int naux, int norb, int fold, int ngroups, int g0, int gcnt,
                                int ldk, const int* __restrict__ ex, const int* __restrict__ ey,
                                unsigned char* __restrict__ X, unsigned char* __restrict__ Y) {
  // groups g0 .. g0 + gcnt - 1 of every instance: planes [4][ninst][gcnt][norb][fold * ldk]
  const int slots = gcnt * fold;
  const int cpr = ldk >> 4;                                       // chunks per row
  const long long items = (long long)ninst * slots * norb * cpr;
  const long long rowlen = (long long)fold * ldk;                 // bytes of a row of X^g
  const long long plane = (long long)ninst * gcnt * norb * rowlen;
  const long long nwave = (long long)gridDim.x * (blockDim.x >> 6);
  const long long wave = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long long span = ((items + nwave - 1) / nwave + 63) / 64 * 64;
  const long long it0 = wave * span + (threadIdx.x & 63);
  const long long it1 = min(items, wave * span + span);
  if (it0 >= it1) return;
  // (instance i, slot P = g fold + seg, row s, chunk c) of item it0
  const long long row0 = it0 / cpr;
  int c = (int)(it0 - row0 * cpr);
  const long long per_inst = (long long)slots * norb;
  int i = (int)(row0 / per_inst);
  const long long rs = row0 - (long long)i * per_inst;
  int P = (int)(rs / norb), s = (int)(rs - (long long)P * norb);
  int g = P / fold, seg = P - g * fold;
  for (long long it = it0; it < it1; it += 64) {
    const long long gr = ((long long)i * ngroups + g0 + g) * norb + s;  // grid: (instance, group, row)
    const int Ex = ex[gr], Ey = ey[gr];
    const int Pg = g0 * fold + P;                                       // the slab
    const bool live = Pg < naux;
    const float* br = b + i * sb + ((long long)(live ? Pg : 0) * norb + s) * norb;
    const float* sr = St + ((long long)i * norb + s) * norb;
    const int q16 = c << 4;
    const long long o = (((long long)i * gcnt + g) * norb + s) * rowlen + (long long)seg * ldk + q16;
    float x[16], y[16];
    if (V4 && live && q16 + 16 <= norb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float4 xv = *(const float4*)(br + q16 + 4 * v), tv = *(const float4*)(sr + q16 + 4 * v);
        x[4 * v] = xv.x; x[4 * v + 1] = xv.y; x[4 * v + 2] = xv.z; x[4 * v + 3] = xv.w;
        y[4 * v] = tv.x * xv.x; y[4 * v + 1] = tv.y * xv.y;
        y[4 * v + 2] = tv.z * xv.z; y[4 * v + 3] = tv.w * xv.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int q = q16 + k;
        x[k] = (live && q < norb) ? br[q] : 0.f;
        y[k] = (live && q < norb) ? sr[q] * x[k] : 0.f;
      }
    }
    i4v px[4], py[4];
    split16_i8(x, Ex, px);
    split16_i8(y, Ey, py);
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      *(i4v*)(X + cc * plane + o) = px[cc];
      *(i4v*)(Y + cc * plane + o) = py[cc];
    }
    // advance by 64 items
    c += 64;
    while (c >= cpr) {
      c -= cpr;
      if (++s == norb) {
        s = 0;
        ++P;
        if (++seg == fold) { seg = 0; ++g; }
        if (P == slots) { P = 0; g = 0; seg = 0; ++i; }
      }
    }
  }
}

long long grid_of(long long items, int per_block) {
  long long g = (items + per_block - 1) / per_block;
  return g < 1 ? 1 : (g > 65536 ? 65536 : g);
}

}  // namespace

int gemm_i8(const I8Desc& d, hipStream_t st) {
  if (d.M < 0 || d.N < 0 || d.K < 0 || d.batch < 0) return NOF_E_DIM;
  if (d.sym && d.M != d.N) return NOF_E_DIM;
  if (d.K > I8_MAX_K) return NOF_E_DIM;
  if (!d.X || !d.Y || !d.ex || !d.ey || (!d.Out && !d.Out64)) return NOF_E_NULL;
  if (d.Out64 && (d.cmax || d.Dg)) return NOF_E_ARG;
  if (d.ldx % IK || d.ldy % IK || d.ldx < d.K || d.ldy < d.K) return NOF_E_DIM;
  if (d.binner < 0 || (d.binner > 0 && (d.cmax || d.batch % d.binner))) return NOF_E_ARG;
  if (d.mslab < 0) return NOF_E_ARG;
  if (d.mslab > 0 && (d.batch != 1 || d.sym || d.Out64 || d.binner || d.mslab < IT || d.M % d.mslab ||
                      (long long)d.M + d.mslab > 0x7fffffffLL))
    return NOF_E_ARG;
  const int tiles_m = (d.M + IT - 1) / IT;
  const int tiles_n = (d.N + IT - 1) / IT;
  const int ntiles = d.sym ? tiles_n * (tiles_n + 1) / 2 : tiles_m * tiles_n;
  const long long G = (long long)ntiles * d.batch;
  if (G <= 0) return NOF_OK;
  if (G > 0x7fffffffLL) return NOF_E_DIM;
  if (d.role == 1)
    hipLaunchKernelGGL(k_transform_stage1_i8, dim3((unsigned)G), dim3(INTHR), 0, st, d, tiles_n, ntiles);
  else if (d.role == 2)
    hipLaunchKernelGGL(k_transform_stage2_i8, dim3((unsigned)G), dim3(INTHR), 0, st, d, tiles_n, ntiles);
  else
    hipLaunchKernelGGL(k_exchange_fock_i8, dim3((unsigned)G), dim3(INTHR), 0, st, d, tiles_n, ntiles);
  return launch_status();
}

// Slabs per group of the INT8 exchange-type product: as many as keep the
// group's contraction (fold * ldk) within the exact int32 depth.
int i8_exchange_fold(int naux, int norb) {
  const long long f = I8_MAX_K / i8_ldk(norb);
  return (int)(f < 1 ? 1 : (f > naux ? naux : f));
}

namespace {
// Bytes of INT8 planes (X and Y together) held at a time: the groups are
// split and multiplied in chunks of as many groups as fit (at least one).
constexpr size_t I8_EX_PLANE_BUDGET = size_t(8) << 30;

struct I8ExLayout {
  int fold, ngroups, gchunk;
  size_t off_mx, off_my, off_ex, off_ey, off_X, off_Y, total;
};
I8ExLayout i8_ex_layout(int ninst, int naux, int norb) {
  I8ExLayout L;
  L.fold = i8_exchange_fold(naux, norb);
  L.ngroups = (naux + L.fold - 1) / L.fold;
  const size_t rows = (size_t)ninst * naux * norb;
  const size_t grows = (size_t)ninst * L.ngroups * norb;
  const size_t per_group = 2 * 4 * (size_t)ninst * norb * (size_t)L.fold * i8_ldk(norb);
  size_t gc = I8_EX_PLANE_BUDGET / per_group;
  L.gchunk = (int)(gc < 1 ? 1 : (gc > (size_t)L.ngroups ? (size_t)L.ngroups : gc));
  const size_t planes = per_group / 2 * L.gchunk;
  L.off_mx = 0;
  L.off_my = align256(L.off_mx + rows * 4);
  L.off_ex = align256(L.off_my + rows * 4);
  L.off_ey = align256(L.off_ex + grows * 4);
  L.off_X = align256(L.off_ey + grows * 4);
  L.off_Y = align256(L.off_X + planes);
  L.total = align256(L.off_Y + planes);
  return L;
}
}  // namespace

size_t i8_exchange_ws(int ninst, int naux, int norb) { return i8_ex_layout(ninst, naux, norb).total; }

int i8_exchange(int ninst, int naux, int norb, const float* b, long long sb, const float* St, double* Out,
                void* ws, hipStream_t st) {
  if (ninst < 1 || naux < 1 || norb < 1) return NOF_E_DIM;
  const I8ExLayout L = i8_ex_layout(ninst, naux, norb);
  char* w = (char*)ws;
  float* mx = (float*)(w + L.off_mx);
  float* my = (float*)(w + L.off_my);
  int* ex = (int*)(w + L.off_ex);
  int* ey = (int*)(w + L.off_ey);
  unsigned char* X = (unsigned char*)(w + L.off_X);
  unsigned char* Y = (unsigned char*)(w + L.off_Y);
  const int ldk = (int)i8_ldk(norb);
  const long long rows = (long long)ninst * naux * norb;
  const bool v4 = norb % 4 == 0 && sb % 4 == 0 && ((size_t)b & 15) == 0 && ((size_t)St & 15) == 0;
  if (v4)
    hipLaunchKernelGGL(k_exch_rowmax_i8<true>, dim3((unsigned)grid_of(rows, 16)), dim3(256), 0, st, b, sb, St,
                       ninst, naux, norb, mx, my);
  else
    hipLaunchKernelGGL(k_exch_rowmax_i8<false>, dim3((unsigned)grid_of(rows, 16)), dim3(256), 0, st, b, sb, St,
                       ninst, naux, norb, mx, my);
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  const long long grows = (long long)ninst * L.ngroups * norb;
  hipLaunchKernelGGL(k_exch_grids_i8, dim3((unsigned)grid_of(grows, 256)), dim3(256), 0, st, mx, my, ninst,
                     naux, norb, L.fold, L.ngroups, ex, ey);
  if ((rc = launch_status()) != NOF_OK) return rc;
  const long long rowlen = (long long)L.fold * ldk;
  const long long n2 = (long long)norb * norb;
  for (int g0 = 0; g0 < L.ngroups; g0 += L.gchunk) {
    const int gc = min(L.gchunk, L.ngroups - g0);
    const long long sitems = (long long)ninst * gc * L.fold * norb * (ldk / 16);
    if (v4)
      hipLaunchKernelGGL(k_exch_split_i8<true>, dim3((unsigned)grid_of(sitems, 256)), dim3(256), 0, st, b, sb,
                         St, ninst, naux, norb, L.fold, L.ngroups, g0, gc, ldk, ex, ey, X, Y);
    else
      hipLaunchKernelGGL(k_exch_split_i8<false>, dim3((unsigned)grid_of(sitems, 256)), dim3(256), 0, st, b, sb,
                         St, ninst, naux, norb, L.fold, L.ngroups, g0, gc, ldk, ex, ey, X, Y);
    if ((rc = launch_status()) != NOF_OK) return rc;
    I8Desc d{};
    d.M = norb; d.N = norb; d.K = (int)rowlen; d.batch = ninst * gc;
    d.binner = ninst > 1 ? gc : 0;
    const long long gstride = (long long)norb * rowlen;              // one group's rows
    const long long plane = (long long)ninst * gc * gstride;
    d.X = X; d.ldx = rowlen; d.sx = gstride; d.sx2 = (long long)gc * gstride; d.psx = plane;
    d.ex = ex + (long long)g0 * norb; d.sex = norb; d.sex2 = (long long)L.ngroups * norb;
    d.Y = Y; d.ldy = rowlen; d.sy = gstride; d.sy2 = (long long)gc * gstride; d.psy = plane;
    d.ey = ey + (long long)g0 * norb; d.sey = norb; d.sey2 = (long long)L.ngroups * norb;
    d.Out64 = Out + (long long)g0 * n2; d.ldo = norb; d.so = n2; d.so2 = (long long)L.ngroups * n2;
    d.sym = false; d.role = 3;
    if ((rc = gemm_i8(d, st)) != NOF_OK) return rc;
  }
  return NOF_OK;
}

int i8_split_rows(const void* A, int At, long long nrow, int K, int ldk, void* planes, int* e,
                  hipStream_t st) {
  if (nrow <= 0 || K <= 0 || ldk < K || ldk % IK) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_of(nrow, 4);
  if (At == NOF_F64)
    hipLaunchKernelGGL(k_split_rows_i8<double>, dim3(g), dim3(256), 0, st, (const double*)A, nrow, K, ldk,
                       (unsigned char*)planes, e);
  else if (At == NOF_F32)
    hipLaunchKernelGGL(k_split_rows_i8<float>, dim3(g), dim3(256), 0, st, (const float*)A, nrow, K, ldk,
                       (unsigned char*)planes, e);
  else
    return NOF_E_DTYPE;
  return launch_status();
}

int i8_split_cols(const double* A, int K, int ncol, int lda, int ldk, void* planes, int* e,
                  hipStream_t st) {
  if (K <= 0 || ncol <= 0 || ldk < K || ldk % IK) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_of(ncol, 16);
  hipLaunchKernelGGL(k_split_cols_i8, dim3(g), dim3(256), 0, st, A, K, ncol, lda, ldk,
                     (unsigned char*)planes, e);
  return launch_status();
}

int i8_cmax_exps(const unsigned* cmax, int batch, int tiles, int N, int* e, hipStream_t st, int mslab) {
  if (batch <= 0 || tiles <= 0 || N <= 0 || mslab < 0 || (mslab > 0 && mslab < IT)) return NOF_E_DIM;
  const unsigned g = (unsigned)grid_of((long long)batch * N, 256);
  hipLaunchKernelGGL(k_cmax_exps_i8, dim3(g), dim3(256), 0, st, cmax, (long long)batch, tiles, N, e, mslab);
  return launch_status();
}

int i8_split_T(const float* T, int batch, int K, int N, long long sT, int ldk, const int* e, void* planes,
               hipStream_t st, long long ldt) {
  if (batch <= 0 || K <= 0 || N <= 0 || ldk < K || ldk % IK || ldt < 0 || (ldt > 0 && ldt < N))
    return NOF_E_DIM;
  const long long blocks = (long long)batch * ((N + 63) / 64) * ((ldk + 127) / 128);
  const unsigned g = (unsigned)(blocks < 1 ? 1 : (blocks > (1 << 20) ? (1 << 20) : blocks));
  hipLaunchKernelGGL(k_split_T_i8, dim3(g), dim3(256), 0, st, T, (long long)batch, K, N, sT, ldt > 0 ? ldt : N,
                     ldk, e, (unsigned char*)planes);
  return launch_status();
}

// Grids of the rows of the per-q products of the exchange-type term: for
// every (q, r), e[q*norb + r] from max_P |b^P[q][r]| (FP32 b [naux][norb][norb]);
// lanes along r, so each slab's row is read coalesced.
__global__ void k_slab_grids_i8(const float* __restrict__ b, int naux, int norb, int* __restrict__ e) {
  const long long n2 = (long long)norb * norb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    unsigned m = 0;
    const float* p = b + i;
#pragma unroll 4
    for (int P = 0; P < naux; ++P) m = max(m, __float_as_uint(p[(long long)P * n2]) & 0x7fffffffu);
    e[i] = grid_exp_i8_bits(m);
  }
}

int i8_slab_grids(const float* b, int naux, int norb, int* e, hipStream_t st) {
  if (naux <= 0 || norb <= 0) return NOF_E_DIM;
  const long long n2 = (long long)norb * norb;
  hipLaunchKernelGGL(k_slab_grids_i8, dim3((unsigned)grid_of(n2, 256)), dim3(256), 0, st, b, naux, norb, e);
  return launch_status();
}

}  // namespace nof
