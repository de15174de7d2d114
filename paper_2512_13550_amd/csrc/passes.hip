// Bandwidth-bound and small FP64 kernels of the JK / generalized-Fock build.
#include "common.h"

namespace nof {
namespace {

// ---------------------------------------------------------------------------
// Exchange and Coulomb-type pass over the unique half of b.
//
// Tile = 16 rows (r) x 128 columns (s) of the norb x norb plane; one
// workgroup walks one tile through a contiguous chunk of auxiliary slabs P.
// Wave w owns rows r = tile_row*16 + 4w + {0..3} (wave-uniform) and lane l
// the columns s = tile_col*128 + 2l + {0,1}; each row is fetched as one
// 2-element vector per lane, so a wave reads 1 KiB contiguous per row and
// slab.  KF_U slabs are in flight per iteration.
//
// The loop is branch-free: a lane whose pair lies outside r <= s (or outside
// the plane) loads a clamped address inside the same row near the diagonal,
// whose cache line the active lanes fetch anyway, and the value is zeroed by
// a select.  W[P][r] is wave-uniform (scalar loads); W[P][s] is one vector
// load per lane.  Tiles strictly inside the upper triangle skip the selects.
// ---------------------------------------------------------------------------
constexpr int KF_R = 16, KF_C = 128, KF_THR = 256, KF_U = 4, KF_RW = 4;
constexpr int KF_GRID64 = 256;   // workgroups of a pass over FP64 b: one per CU
constexpr int KF_MAXCHUNK = 64;  // partial planes at most
constexpr int KF_MINSLABS = 16;  // slabs per chunk at least (small naux)
constexpr int KF_PIPE = 1;       // slab loop: 0 groups of KF_U, 1 double-buffered

__device__ __forceinline__ void kf_tile(int t, int ntc, int ntr, int& tr, int& tc) {
  // tiles are listed column-block by column-block; column block tc holds the
  // row blocks 0 .. min(ntr, (tc*128+127)/16 + 1) - 1 (those touching r <= s)
  for (tc = 0; tc < ntc; ++tc) {
    int cnt = (tc * KF_C + KF_C - 1) / KF_R + 1;
    if (cnt > ntr) cnt = ntr;
    if (t < cnt) { tr = t; return; }
    t -= cnt;
  }
  tr = -1;
}

template <typename TB> struct Vec2;
template <> struct Vec2<double> { typedef double2 t; };
template <> struct Vec2<float> { typedef float2 t; };

// Per-lane state of one tile: the clamped (wave-uniform) row offsets and
// per-lane columns of the loads, the select masks and the clamped W indices.
struct KfLane {
  long long roff[KF_RW];  // rr * norb, rr = clamped row (wave-uniform)
  int col[KF_RW][2];      // clamped columns of the pair
  bool act[KF_RW][2];
  int wl;                 // clamped row r0 + (lane mod KF_RW), read into wl
  int ws;                 // clamped column index of the pair's first column
};

// One slab's operands of a lane: the pair of every row, and for the
// Coulomb-type term W[P][s], W[P][s+1] and wl = W[P][row (lane mod KF_RW)] of
// the wave's rows (lanes 0 .. KF_RW-1 hold the KF_RW row values, which every
// lane reads back with readlane: one vector load instead of one per row).
template <typename TB> struct KfSlab {
  TB v[KF_RW][2];
  double ws0, ws1, wl;
};

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long x = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)x, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename TB, bool VEC, bool FULL, bool wantF, int PIPE>
__device__ __forceinline__ void kf_run(const TB* __restrict__ b, const double* __restrict__ W,
                                       int norb, long long plane, int p_lo, int p_hi,
                                       const KfLane& L, double (&k)[KF_RW][2],
                                       double (&frs)[KF_RW][2], double (&fsr)[KF_RW][2]) {
  typedef typename Vec2<TB>::t V2;
  // every load of a slab (b and W) is issued before any of its values is used
  auto fetch = [&](int P, KfSlab<TB>& x) {
    const TB* pl = b + (long long)P * plane;
#pragma unroll
    for (int i = 0; i < KF_RW; ++i) {
      const TB* row = pl + L.roff[i];
      if (VEC) {
        const V2 t = *(const V2*)(row + L.col[i][0]);
        x.v[i][0] = t.x;
        x.v[i][1] = t.y;
      } else {
        x.v[i][0] = row[L.col[i][0]];
        x.v[i][1] = row[L.col[i][1]];
      }
    }
    if (wantF) {
      const double* wp = W + (long long)P * norb;
      if (VEC) {
        const double2 t = *(const double2*)(wp + L.ws);
        x.ws0 = t.x;
        x.ws1 = t.y;
      } else {
        x.ws0 = wp[L.ws];
        x.ws1 = wp[L.ws + 1 < norb ? L.ws + 1 : L.ws];
      }
      x.wl = wp[L.wl];
    }
  };
  auto accum = [&](KfSlab<TB>& x) {
    double wr[KF_RW];
    if (wantF) {
#pragma unroll
      for (int i = 0; i < KF_RW; ++i) wr[i] = readlane_f64(x.wl, i);
    }
#pragma unroll
    for (int i = 0; i < KF_RW; ++i) {
      double a0 = (double)x.v[i][0], a1 = (double)x.v[i][1];
      if (!FULL) {
        a0 = L.act[i][0] ? a0 : 0.0;
        a1 = L.act[i][1] ? a1 : 0.0;
      }
      k[i][0] = fma(a0, a0, k[i][0]);
      k[i][1] = fma(a1, a1, k[i][1]);
      if (wantF) {
        frs[i][0] = fma(a0, x.ws0, frs[i][0]);
        frs[i][1] = fma(a1, x.ws1, frs[i][1]);
        fsr[i][0] = fma(a0, wr[i], fsr[i][0]);
        fsr[i][1] = fma(a1, wr[i], fsr[i][1]);
      }
    }
  };
  if (PIPE == 0) {
    // groups of KF_U slabs: all loads of a group issued, then all used
    int P = p_lo;
    for (; P + KF_U <= p_hi; P += KF_U) {
      KfSlab<TB> x[KF_U];
#pragma unroll
      for (int u = 0; u < KF_U; ++u) fetch(P + u, x[u]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < KF_U; ++u) accum(x[u]);
    }
    for (; P < p_hi; ++P) {
      KfSlab<TB> x;
      fetch(P, x);
      accum(x);
    }
  } else {
    // double-buffered: slab P+1 in flight while slab P is used
    if (p_lo >= p_hi) return;
    KfSlab<TB> x, y;
    fetch(p_lo, x);
    int P = p_lo;
    for (; P + 2 <= p_hi; P += 2) {
      fetch(P + 1, y);
      __builtin_amdgcn_sched_barrier(0);
      accum(x);
      if (P + 2 < p_hi) fetch(P + 2, x);
      __builtin_amdgcn_sched_barrier(0);
      accum(y);
    }
    if (P < p_hi) accum(x);
  }
}

// Work units: (instance, chunk of slabs, tile), tile fastest.  The grid
// sweeps the units in order, unit u on workgroup u mod G, so the workgroups
// of one sweep read all tiles of the same few slabs at the same time (whole
// planes read densely) and each workgroup gets the same number of units.
// Unit (i, c, t) writes plane c of instance i's partials; a chunk past the
// last slab writes zeros, so summing the nchunk planes in order gives the
// sums over all slabs (fixed order, no atomics).
//
// VEC: norb even and b 16-byte aligned, so every pair starting at an even
// column is one aligned vector.  Instance i reads b + i*bstride, W + i*wstride
// and writes its partials at + i*pstride.
template <typename TB, bool VEC, int PIPE, bool WANTF>
__global__ __launch_bounds__(KF_THR) void k_kf1(int naux, int norb, const TB* __restrict__ b,
                                                const double* __restrict__ W,
                                                double* __restrict__ Kpart,
                                                double* __restrict__ F1part, int pchunk,
                                                int nchunk, int ntiles, int ntr, int ntc,
                                                int ninst, long long bstride, long long wstride,
                                                long long pstride) {
  const long long units = (long long)ninst * nchunk * ntiles;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const long long plane = (long long)norb * norb;
  constexpr bool wantF = WANTF;
  for (long long u = blockIdx.x; u < units; u += gridDim.x) {
    const int tile = (int)(u % ntiles);
    const long long ic = u / ntiles;
    const int chunk = (int)(ic % nchunk);
    const int inst = (int)(ic / nchunk);
    const int p_lo = min(naux, chunk * pchunk);
    const int p_hi = min(naux, p_lo + pchunk);
    const TB* bi = b + (long long)inst * bstride;
    const double* Wi = W ? W + (long long)inst * wstride : nullptr;
    int tr, tc;
    kf_tile(tile, ntc, ntr, tr, tc);
    const int s0 = tc * KF_C + 2 * lane;
    const int r0 = tr * KF_R + wv * KF_RW;

    KfLane L;
#pragma unroll
    for (int i = 0; i < KF_RW; ++i) {
      const int r = r0 + i;
      const int rr = min(r, norb - 1);
      L.roff[i] = (long long)rr * norb;
#pragma unroll
      for (int c = 0; c < 2; ++c) L.act[i][c] = (s0 + c < norb) && (r < norb) && (r <= s0 + c);
      if (VEC) {
        // the pair (cc, cc+1), cc even, cc <= norb-2, never left of the
        // diagonal pair of row rr
        L.col[i][0] = min(max(s0, rr & ~1), norb - 2);
        L.col[i][1] = L.col[i][0] + 1;
      } else {
#pragma unroll
        for (int c = 0; c < 2; ++c) L.col[i][c] = min(max(s0 + c, rr), norb - 1);
      }
    }
    L.ws = VEC ? min(s0, norb - 2) : min(s0, norb - 1);
    L.wl = min(r0 + (lane & (KF_RW - 1)), norb - 1);
    // tile strictly inside r <= s and inside the plane: no lane is masked
    const bool full = (tr * KF_R + KF_R - 1 <= tc * KF_C) && (tc * KF_C + KF_C <= norb) &&
                      (tr * KF_R + KF_R <= norb);

    double k[KF_RW][2] = {}, frs[KF_RW][2] = {}, fsr[KF_RW][2] = {};
    if (full)
      kf_run<TB, VEC, true, WANTF, PIPE>(bi, Wi, norb, plane, p_lo, p_hi, L, k, frs, fsr);
    else
      kf_run<TB, VEC, false, WANTF, PIPE>(bi, Wi, norb, plane, p_lo, p_hi, L, k, frs, fsr);

    const long long cb = (long long)inst * pstride + (long long)chunk * plane;
#pragma unroll
    for (int i = 0; i < KF_RW; ++i)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (!L.act[i][c]) continue;
        const int r = r0 + i, s = s0 + c;
        if (Kpart) Kpart[cb + (long long)r * norb + s] = k[i][c];
        if (wantF) {
          F1part[cb + (long long)r * norb + s] = frs[i][c];
          if (r != s) F1part[cb + (long long)s * norb + r] = fsr[i][c];
        }
      }
  }
}

__global__ void k_reduce(const double* __restrict__ part, int nparts, long long stride, int norb,
                         int sym_upper, double* __restrict__ out, long long pinst, long long oinst) {
  const long long n2 = (long long)norb * norb;
  part += (long long)blockIdx.y * pinst;
  out += (long long)blockIdx.y * oinst;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    long long src = i;
    if (sym_upper) {
      const int r = (int)(i / norb), s = (int)(i - (long long)r * norb);
      src = r <= s ? i : (long long)s * norb + r;
    }
    double a = 0.0;
    for (int c = 0; c < nparts; ++c) a += part[(long long)c * stride + src];
    out[i] = a;
  }
}

// Exchange-type term from the per-q symmetric products G^q (FP64):
//   F[r][s] = start[r][s] + sum_{q < qn} cK[q][s] G[q][r][s]
// summed in q order; start = F (mode 1), -F1 (mode 2) or 0 (mode 0).  One
// thread per element (r, s): the loads of G and cK run along s (coalesced).
// Instance blockIdx.y at G + y*gstride, cK + y*cstride, F1 and F + y*fstride.
__global__ void k_exchange_accum(const double* __restrict__ G, int qn, int norb,
                                 const double* __restrict__ cK, const double* __restrict__ F1, int mode,
                                 double* __restrict__ F, long long gstride, long long cstride,
                                 long long fstride) {
  const long long n2 = (long long)norb * norb;
  G += blockIdx.y * gstride;
  cK += blockIdx.y * cstride;
  F += blockIdx.y * fstride;
  if (F1) F1 += blockIdx.y * fstride;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(i % norb);
    double a = mode == 1 ? F[i] : (mode == 2 ? -F1[i] : 0.0);
#pragma unroll 4
    for (int q = 0; q < qn; ++q) a = fma(cK[(long long)q * norb + s], G[(long long)q * n2 + i], a);
    F[i] = a;
  }
}

// y -= x over n elements.
__global__ void k_subtract(long long n, const double* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] -= x[i];
}

__global__ void k_lambda(int norb, const double* __restrict__ n, const double* __restrict__ h,
                         const double* __restrict__ F1, const double* __restrict__ F2,
                         double* __restrict__ lam, double* __restrict__ grad, long long nstride,
                         long long mstride, long long fstride) {
  const long long n2 = (long long)norb * norb;
  const long long y = blockIdx.y;
  n += y * nstride;
  h += y * mstride;
  lam += y * mstride;
  if (grad) grad += y * mstride;
  // F1 == NULL: F2 already holds the exchange-type minus the Coulomb-type term
  if (F1) F1 += y * fstride;
  F2 += y * fstride;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / norb), s = (int)(i - (long long)r * norb);
    const long long t = (long long)s * norb + r;
    const double l_rs = F1 ? n[s] * h[i] + F1[i] - F2[i] : n[s] * h[i] - F2[i];
    lam[i] = l_rs;
    if (grad) {
      const double l_sr = F1 ? n[r] * h[t] + F1[t] - F2[t] : n[r] * h[t] - F2[t];
      grad[i] = 4.0 * (l_rs - l_sr);
    }
  }
}

// Energy in two fixed-order steps (bitwise repeatable): workgroup c of
// instance y sums elements [c*chunk, (c+1)*chunk) of cJ o J - cK o K and the
// diagonal terms 2 n_p h_pp of its share of p into part[y*E_PARTS + c]; one
// workgroup per instance then adds the E_PARTS partials in a fixed tree.
constexpr int E_PARTS = 128, E_THR = 256;
__global__ __launch_bounds__(E_THR) void k_energy_part(int norb, const double* __restrict__ n,
                                                       const double* __restrict__ h,
                                                       const double* __restrict__ J,
                                                       const double* __restrict__ K,
                                                       const double* __restrict__ cJ,
                                                       const double* __restrict__ cK,
                                                       double* __restrict__ part, long long nstride,
                                                       long long mstride, long long jstride) {
  __shared__ double red[E_THR];
  const long long n2 = (long long)norb * norb;
  const long long y = blockIdx.y;
  const int c = blockIdx.x;
  n += y * nstride;
  h += y * mstride;
  cJ += y * mstride;
  cK += y * mstride;
  J += y * jstride;
  K += y * jstride;
  const long long chunk = (n2 + E_PARTS - 1) / E_PARTS;
  const long long lo = c * chunk, hi = min(n2, lo + chunk);
  double a = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += E_THR) a += cJ[i] * J[i] - cK[i] * K[i];
  const int pc = (norb + E_PARTS - 1) / E_PARTS;
  const int p_hi = min(norb, (c + 1) * pc);
  for (int p = c * pc + threadIdx.x; p < p_hi; p += E_THR) a += 2.0 * n[p] * h[(long long)p * norb + p];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = E_THR / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[y * E_PARTS + c] = red[0];
}

__global__ __launch_bounds__(E_PARTS) void k_energy_sum(const double* __restrict__ part,
                                                        double* __restrict__ E) {
  __shared__ double red[E_PARTS];
  const long long y = blockIdx.x;
  red[threadIdx.x] = part[y * E_PARTS + threadIdx.x];
  __syncthreads();
  for (int w = E_PARTS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) E[y] = red[0];
}

__global__ void k_coeffs(int norb, const double* __restrict__ n, const double* __restrict__ Delta,
                         const double* __restrict__ Pi, double* __restrict__ cJ,
                         double* __restrict__ cK) {
  const long long n2 = (long long)norb * norb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i / norb), q = (int)(i - (long long)p * norb);
    const double nn = n[p] * n[q];
    const double d = Delta ? Delta[i] : 0.0;
    const double pi = Pi ? Pi[i] : 0.0;
    cJ[i] = 2.0 * (nn - d);
    cK[i] = nn - d - pi;
  }
}

inline int grid_for(long long n, int thr) {
  long long g = (n + thr - 1) / thr;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

void kf_geometry(int norb, int& ntr, int& ntc, int& ntiles) {
  ntr = (norb + KF_R - 1) / KF_R;
  ntc = (norb + KF_C - 1) / KF_C;
  ntiles = 0;
  for (int tc = 0; tc < ntc; ++tc) {
    int cnt = (tc * KF_C + KF_C - 1) / KF_R + 1;
    ntiles += cnt > ntr ? ntr : cnt;
  }
}


// Plan of one pass: nchunk chunks of pchunk slabs, G workgroups.  With few
// units per CU the slowest CU sets the time, so the chunk count is the
// smallest whose units fill the grid (KF_GRID64 workgroups for FP64 b, twice
// that for FP32 b, whose waves hold half the bytes in flight) to within 7 %;
// with at least 8 units per workgroup the grid is one workgroup per unit and
// the hardware balances it.
struct KfPlan {
  int nchunk, pchunk, G;
};

KfPlan kf_plan(int naux, int norb, int ninst, int bt) {
  int ntr, ntc, ntiles;
  kf_geometry(norb, ntr, ntc, ntiles);
  const long long grid = bt == NOF_F64 ? KF_GRID64 : 2 * KF_GRID64;
  const long long per = (long long)ninst * ntiles;
  int ncmax = naux / KF_MINSLABS < KF_MAXCHUNK ? naux / KF_MINSLABS : KF_MAXCHUNK;
  if (ncmax < 1) ncmax = 1;
  int nc = ncmax;
  for (int c = 1; c <= ncmax; ++c) {
    const long long units = per * c;
    if (units >= 8 * grid) { nc = c; break; }
    const long long rounds = (units + grid - 1) / grid;
    if (units * 10 >= grid * 9 && rounds * grid * 100 <= units * 107) { nc = c; break; }
  }
  KfPlan pl;
  pl.pchunk = (naux + nc - 1) / nc;
  pl.nchunk = (naux + pl.pchunk - 1) / pl.pchunk;
  const long long units = per * pl.nchunk;
  long long G = units >= 8 * grid || units < grid ? units : grid;
  if (G > (1 << 24)) G = 1 << 24;  // the workgroups sweep the units in any case
  pl.G = (int)G;
  return pl;
}

}  // namespace

int kf1_parts(int naux, int norb, int ninst, int bt) { return kf_plan(naux, norb, ninst, bt).nchunk; }

int kf1_pass(int naux, int norb, const void* b, int bt, const double* W, double* Kpart,
             double* F1part, int nparts, hipStream_t st, int ninst, long long bstride,
             long long wstride, long long pstride) {
  if (ninst < 1 || ninst > 65535) return NOF_E_DIM;
  int ntr, ntc, ntiles;
  kf_geometry(norb, ntr, ntc, ntiles);
  const KfPlan pl = kf_plan(naux, norb, ninst, bt);
  if (nparts != pl.nchunk) return NOF_E_INTERNAL;
  if (ninst > 1 && pstride < (long long)nparts * norb * norb) return NOF_E_INTERNAL;
  const dim3 grid((unsigned)pl.G);
  const size_t esz = bt == NOF_F64 ? 8 : 4;
  const bool vec = (norb % 2) == 0 && ((uintptr_t)b % 16) == 0 && ((bstride * esz) % 16) == 0 &&
                   (!W || (((uintptr_t)W % 16) == 0 && (wstride % 2) == 0));
#define NOF_KF1(TB, V)                                                                          \
  do {                                                                                          \
    if (F1part)                                                                                 \
      hipLaunchKernelGGL((k_kf1<TB, V, KF_PIPE, true>), grid, dim3(KF_THR), 0, st, naux, norb,  \
                         (const TB*)b, W, Kpart, F1part, pl.pchunk, pl.nchunk, ntiles, ntr, ntc, \
                         ninst, bstride, wstride, pstride);                                     \
    else                                                                                        \
      hipLaunchKernelGGL((k_kf1<TB, V, KF_PIPE, false>), grid, dim3(KF_THR), 0, st, naux, norb, \
                         (const TB*)b, W, Kpart, F1part, pl.pchunk, pl.nchunk, ntiles, ntr, ntc, \
                         ninst, bstride, wstride, pstride);                                     \
  } while (0)
  if (bt == NOF_F64) {
    if (vec) NOF_KF1(double, true); else NOF_KF1(double, false);
  } else if (bt == NOF_F32) {
    if (vec) NOF_KF1(float, true); else NOF_KF1(float, false);
  } else {
    return NOF_E_DTYPE;
  }
#undef NOF_KF1
  return launch_status();
}

int reduce_parts(const double* part, int nparts, long long stride, int norb, bool sym_upper,
                 double* out, hipStream_t st, int ninst, long long pinst, long long oinst) {
  const long long n2 = (long long)norb * norb;
  hipLaunchKernelGGL(k_reduce, dim3(grid_for(n2, 256), ninst), dim3(256), 0, st, part, nparts,
                     stride, norb, sym_upper ? 1 : 0, out, pinst, oinst);
  return launch_status();
}

int lambda_grad(int norb, const double* n, const double* h, const double* F1, const double* F2,
                double* lam, double* grad, hipStream_t st, int ninst, long long nstride,
                long long mstride, long long fstride) {
  const long long n2 = (long long)norb * norb;
  hipLaunchKernelGGL(k_lambda, dim3(grid_for(n2, 256), ninst), dim3(256), 0, st, norb, n, h, F1,
                     F2, lam, grad, nstride, mstride, fstride);
  return launch_status();
}

int exchange_accum(const double* G, int qn, int norb, const double* cK, const double* F1, int mode,
                   double* F, hipStream_t st, int ninst, long long gstride, long long cstride,
                   long long fstride) {
  if (qn < 1 || norb < 1 || ninst < 1 || ninst > 65535 || mode < 0 || mode > 2 || (mode == 2 && !F1))
    return NOF_E_ARG;
  const long long n2 = (long long)norb * norb;
  hipLaunchKernelGGL(k_exchange_accum, dim3(grid_for(n2, 256), ninst), dim3(256), 0, st, G, qn, norb, cK, F1,
                     mode, F, gstride, cstride, fstride);
  return launch_status();
}

int subtract(long long n, const double* x, double* y, hipStream_t st, int ninst, long long xstride,
             long long ystride) {
  for (int i = 0; i < ninst; ++i) {
    hipLaunchKernelGGL(k_subtract, dim3(grid_for(n, 256)), dim3(256), 0, st, n, x + i * xstride,
                       y + i * ystride);
    const int rc = launch_status();
    if (rc != NOF_OK) return rc;
  }
  return NOF_OK;
}

size_t energy_ws(int ninst) { return align256((size_t)ninst * E_PARTS * sizeof(double)); }

int energy(int norb, const double* n, const double* h, const double* J, const double* K,
           const double* cJ, const double* cK, double* E, double* part, hipStream_t st, int ninst,
           long long nstride, long long mstride, long long jstride) {
  hipLaunchKernelGGL(k_energy_part, dim3(E_PARTS, ninst), dim3(E_THR), 0, st, norb, n, h, J, K, cJ,
                     cK, part, nstride, mstride, jstride);
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  hipLaunchKernelGGL(k_energy_sum, dim3(ninst), dim3(E_PARTS), 0, st, part, E);
  return launch_status();
}

int coeffs_from_cumulant(int norb, const double* n, const double* Delta, const double* Pi,
                         double* cJ, double* cK, hipStream_t st) {
  const long long n2 = (long long)norb * norb;
  hipLaunchKernelGGL(k_coeffs, dim3(grid_for(n2, 256)), dim3(256), 0, st, norb, n, Delta, Pi, cJ,
                     cK);
  return launch_status();
}

}  // namespace nof
