// Bandwidth-bound and small FP64 kernels of the JK / generalized-Fock build.
#include "common.h"

namespace nof {
namespace {

// ---------------------------------------------------------------------------
// Exchange and Coulomb-type pass over the unique half of b.
//
// Tile = 16 rows (r) x 128 columns (s) of the norb x norb plane; one
// workgroup walks one tile through a contiguous chunk of auxiliary slabs P.
// Thread (ty, tx) owns columns s = tile_col*128 + 2*tx + {0,1} and rows
// r = tile_row*16 + 4*ty + {0..3}; each row is fetched as one 2-element vector
// (16 B in FP64), so a wave reads 1 KiB contiguous per row and slab.  Four
// slabs are in flight per iteration.  W (naux x norb, FP64) is L2 resident.
// ---------------------------------------------------------------------------
constexpr int KF_R = 16, KF_C = 128, KF_THR = 256, KF_U = 4;

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

// VEC: norb even, so every row segment starting at an even column is aligned.
// Instance i (blockIdx.y) reads b + i*bstride, W + i*wstride and writes its
// partials at + i*pstride.
template <typename TB, bool VEC>
__global__ __launch_bounds__(KF_THR) void k_kf1(int naux, int norb, const TB* __restrict__ b,
                                                const double* __restrict__ W,
                                                double* __restrict__ Kpart,
                                                double* __restrict__ F1part, int pchunk,
                                                int ntiles, int ntr, int ntc, long long bstride,
                                                long long wstride, long long pstride) {
  typedef typename Vec2<TB>::t V2;
  const int tile = blockIdx.x % ntiles;
  const int chunk = blockIdx.x / ntiles;
  b += (long long)blockIdx.y * bstride;
  if (W) W += (long long)blockIdx.y * wstride;
  if (Kpart) Kpart += (long long)blockIdx.y * pstride;
  if (F1part) F1part += (long long)blockIdx.y * pstride;
  int tr, tc;
  kf_tile(tile, ntc, ntr, tr, tc);
  if (tr < 0) return;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int s0 = tc * KF_C + 2 * tx;
  const int r0 = tr * KF_R + ty * 4;
  const int p_lo = chunk * pchunk;
  const int p_hi = min(naux, p_lo + pchunk);
  const long long plane = (long long)norb * norb;
  const bool wantF = F1part != nullptr;

  bool act[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c)
      act[i][c] = (s0 + c < norb) && (r0 + i < norb) && (r0 + i <= s0 + c);
  bool rowany[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) rowany[i] = act[i][0] || act[i][1];

  double k[4][2] = {}, frs[4][2] = {}, fsr[4][2] = {};

  auto fetch = [&](int P, int i, TB& v0, TB& v1) {
    const TB* row = b + (long long)P * plane + (long long)(r0 + i) * norb + s0;
    if (VEC) {
      V2 v = rowany[i] ? *(const V2*)row : V2{0, 0};
      v0 = act[i][0] ? v.x : (TB)0;
      v1 = act[i][1] ? v.y : (TB)0;
    } else {
      v0 = act[i][0] ? row[0] : (TB)0;
      v1 = act[i][1] ? row[1] : (TB)0;
    }
  };
  auto accum = [&](int P, const TB (&v)[4][2]) {
    double ws0 = 0.0, ws1 = 0.0, wr[4] = {0, 0, 0, 0};
    if (wantF) {
      const double* wp = W + (long long)P * norb;
      ws0 = s0 < norb ? wp[s0] : 0.0;
      ws1 = s0 + 1 < norb ? wp[s0 + 1] : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) wr[i] = (r0 + i < norb) ? wp[r0 + i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double a0 = (double)v[i][0], a1 = (double)v[i][1];
      k[i][0] = fma(a0, a0, k[i][0]);
      k[i][1] = fma(a1, a1, k[i][1]);
      if (wantF) {
        frs[i][0] = fma(a0, ws0, frs[i][0]);
        frs[i][1] = fma(a1, ws1, frs[i][1]);
        fsr[i][0] = fma(a0, wr[i], fsr[i][0]);
        fsr[i][1] = fma(a1, wr[i], fsr[i][1]);
      }
    }
  };

  int P = p_lo;
  for (; P + KF_U <= p_hi; P += KF_U) {
    TB v[KF_U][4][2];
#pragma unroll
    for (int u = 0; u < KF_U; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) fetch(P + u, i, v[u][i][0], v[u][i][1]);
#pragma unroll
    for (int u = 0; u < KF_U; ++u) accum(P + u, v[u]);
  }
  for (; P < p_hi; ++P) {
    TB v[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i) fetch(P, i, v[i][0], v[i][1]);
    accum(P, v);
  }

  const long long cb = (long long)chunk * plane;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!act[i][c]) continue;
      const int r = r0 + i, s = s0 + c;
      if (Kpart) Kpart[cb + (long long)r * norb + s] = k[i][c];
      if (wantF) {
        F1part[cb + (long long)r * norb + s] = frs[i][c];
        if (r != s) F1part[cb + (long long)s * norb + r] = fsr[i][c];
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
  F1 += y * fstride;
  F2 += y * fstride;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / norb), s = (int)(i - (long long)r * norb);
    const long long t = (long long)s * norb + r;
    const double l_rs = n[s] * h[i] + F1[i] - F2[i];
    lam[i] = l_rs;
    if (grad) {
      const double l_sr = n[r] * h[t] + F1[t] - F2[t];
      grad[i] = 4.0 * (l_rs - l_sr);
    }
  }
}

constexpr int E_THR = 1024;
__global__ __launch_bounds__(E_THR) void k_energy(int norb, const double* __restrict__ n,
                                                  const double* __restrict__ h,
                                                  const double* __restrict__ J,
                                                  const double* __restrict__ K,
                                                  const double* __restrict__ cJ,
                                                  const double* __restrict__ cK,
                                                  double* __restrict__ E, long long nstride,
                                                  long long mstride, long long jstride) {
  __shared__ double red[E_THR];
  const long long n2 = (long long)norb * norb;
  const long long y = blockIdx.x;
  n += y * nstride;
  h += y * mstride;
  cJ += y * mstride;
  cK += y * mstride;
  J += y * jstride;
  K += y * jstride;
  E += y;
  double a = 0.0;
  for (long long i = threadIdx.x; i < n2; i += E_THR) a += cJ[i] * J[i] - cK[i] * K[i];
  for (int p = threadIdx.x; p < norb; p += E_THR) a += 2.0 * n[p] * h[(long long)p * norb + p];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = E_THR / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E = red[0];
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

}  // namespace

int kf1_chunks(int naux, int norb) {
  int ntr, ntc, ntiles;
  kf_geometry(norb, ntr, ntc, ntiles);
  int nc = (2048 + ntiles - 1) / ntiles;
  if (nc > naux) nc = naux;
  if (nc < 1) nc = 1;
  return nc;
}

int kf1_pass(int naux, int norb, const void* b, int bt, const double* W, double* Kpart,
             double* F1part, int nchunk, hipStream_t st, int ninst, long long bstride,
             long long wstride, long long pstride) {
  int ntr, ntc, ntiles;
  kf_geometry(norb, ntr, ntc, ntiles);
  const int pchunk = (naux + nchunk - 1) / nchunk;
  const int nc = (naux + pchunk - 1) / pchunk;
  if (nc > nchunk) return NOF_E_INTERNAL;
  const long long G = (long long)ntiles * nchunk;
  if (G > 0x7fffffffLL || ninst < 1 || ninst > 65535) return NOF_E_DIM;
  // chunks beyond nc (when pchunk rounding leaves them empty) write zeros
  const dim3 grid((unsigned)G, (unsigned)ninst);
  const size_t esz = bt == NOF_F64 ? 8 : 4;
  const bool vec = (norb % 2) == 0 && ((uintptr_t)b % 16) == 0 && ((bstride * esz) % 16) == 0;
  if (bt == NOF_F64) {
    if (vec)
      hipLaunchKernelGGL((k_kf1<double, true>), grid, dim3(KF_THR), 0, st, naux, norb,
                         (const double*)b, W, Kpart, F1part, pchunk, ntiles, ntr, ntc, bstride,
                         wstride, pstride);
    else
      hipLaunchKernelGGL((k_kf1<double, false>), grid, dim3(KF_THR), 0, st, naux, norb,
                         (const double*)b, W, Kpart, F1part, pchunk, ntiles, ntr, ntc, bstride,
                         wstride, pstride);
  } else if (bt == NOF_F32) {
    if (vec)
      hipLaunchKernelGGL((k_kf1<float, true>), grid, dim3(KF_THR), 0, st, naux, norb,
                         (const float*)b, W, Kpart, F1part, pchunk, ntiles, ntr, ntc, bstride,
                         wstride, pstride);
    else
      hipLaunchKernelGGL((k_kf1<float, false>), grid, dim3(KF_THR), 0, st, naux, norb,
                         (const float*)b, W, Kpart, F1part, pchunk, ntiles, ntr, ntc, bstride,
                         wstride, pstride);
  } else {
    return NOF_E_DTYPE;
  }
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

int energy(int norb, const double* n, const double* h, const double* J, const double* K,
           const double* cJ, const double* cK, double* E, hipStream_t st, int ninst,
           long long nstride, long long mstride, long long jstride) {
  hipLaunchKernelGGL(k_energy, dim3(ninst), dim3(E_THR), 0, st, norb, n, h, J, K, cJ, cK, E,
                     nstride, mstride, jstride);
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
