// FP64 orbital-rotation step (NO Optimization: U = exp(y) with y
// antisymmetric, C <- C U, and the ADAM update of y from the orbital gradient).
//
// exp(y) is evaluated by scaling and squaring with a degree-12 Taylor
// polynomial (Higham, "The scaling and squaring method for the matrix
// exponential revisited", SIAM J. Matrix Anal. Appl. 26 (2005)): the scaling
// power s is chosen on the device from the Frobenius norm so that
// ||y / 2^s||_F <= 1/4, where the truncation error is below 3e-18; the
// polynomial is evaluated by the Paterson-Stockmeyer scheme (Paterson and
// Stockmeyer, SIAM J. Comput. 2 (1973)) in blocks of four powers,
//   p(x) = B0 + x^4 (B1 + x^4 B2),  B_j = sum_i x^i / (4j + i)!,
// which takes five products (y^2, y^3, y^4 and two by x^4) where Horner's rule
// takes eleven, and the result is then squared s times.  Every
// product is a split-K matrix-core GEMM (the matrices are small, so the K
// dimension is spread over workgroups) followed by a fixed-order combine.  Nothing is read back to the host,
// so the whole step stays asynchronous (and graph capturable): the squaring
// launches beyond s exit immediately.
#include <math.h>

#include <algorithm>

#include "common.h"

namespace nof {
namespace {

constexpr int kTaylor = 12;
constexpr int kMaxSquare = 16;      // ||y||_F up to 2^16 / 4
constexpr double kTheta = 0.25;

struct ExpmScratch {
  int s;
  int pad;
  double scale;   // 2^-s
};

// ||y||_F (a sub-multiplicative norm, so the Taylor truncation bound holds for
// it) -> scaling power s with ||y||_F / 2^s <= 1/4.
// Instance blockIdx.x: y + i*n2 -> sc[i].
__global__ __launch_bounds__(1024) void k_norm_scale(int norb, const double* __restrict__ y,
                                                     ExpmScratch* __restrict__ sc) {
  __shared__ double red[1024];
  const long long n2 = (long long)norb * norb;
  y += blockIdx.x * n2;
  sc += blockIdx.x;
  // eight independent partial sums keep eight loads in flight per thread
  double acc[8] = {};
  long long i = threadIdx.x;
  for (; i + 7 * 1024 < n2; i += 8 * 1024) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = y[i + u * 1024];
    __builtin_amdgcn_sched_barrier(0);    // every load issued before any is used
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = fma(v[u], v[u], acc[u]);
  }
  for (; i < n2; i += 1024) acc[0] = fma(y[i], y[i], acc[0]);
  double a = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) a += acc[u];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nrm = sqrt(red[0]);
    int s = 0;
    double sc_ = 1.0;
    while (nrm * sc_ > kTheta && s < kMaxSquare) { ++s; sc_ *= 0.5; }
    sc->s = s;
    sc->scale = sc_;
  }
}

// Instance i = blockIdx.y: out_i = diag_c * I + coef * sum_c part_i[c] (fixed
// summation order), part_i = part + i*pinst, out_i = out + i*oinst;
// coef = coef_mul * sc[i].scale when sc is given.  With pred_sc the kernel
// runs only when pred_sc[i].s > pred_gt.
__global__ void k_combine(int rows, int cols, const double* __restrict__ part, int nparts,
                          long long stride, double diag_c, double coef_mul,
                          const ExpmScratch* __restrict__ sc, const ExpmScratch* __restrict__ pred_sc,
                          int pred_gt, double* __restrict__ out, long long pinst, long long oinst) {
  const int y = blockIdx.y;
  if (pred_sc && pred_sc[y].s <= pred_gt) return;
  part += y * pinst;
  out += y * oinst;
  const double coef = sc ? coef_mul * sc[y].scale : coef_mul;
  const long long n = (long long)rows * cols;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < nparts; ++c) a += part[(long long)c * stride + i];
    const int r = (int)(i / cols), q = (int)(i - (long long)r * cols);
    out[i] = (r == q ? diag_c : 0.0) + coef * a;
  }
}

// Instance i = blockIdx.y: out_i = add_i + sc[i].scale^4 * sum_c part_i[c]
// (fixed summation order); the Horner step in x^4 = (2^-s y)^4.
__global__ void k_combine_x4(long long n2, const double* __restrict__ part, int nparts, long long stride,
                             const ExpmScratch* __restrict__ sc, const double* __restrict__ add,
                             double* __restrict__ out, long long pinst, long long oinst) {
  const int y = blockIdx.y;
  part += y * pinst;
  add += y * oinst;
  out += y * oinst;
  const double s = sc[y].scale, coef = (s * s) * (s * s);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < nparts; ++c) a += part[(long long)c * stride + i];
    out[i] = add[i] + coef * a;
  }
}

// One block of the Taylor polynomial in x = sc[i].scale * y for instance
// i = blockIdx.y: out = sum_{j<np} c[j] x^j with x^0 = I, x^1 from y and x^2,
// x^3, x^4 from the unscaled powers P2, P3, P4 (np <= 5).
struct TaylorBlock {
  double c[5];
  int np;
};
__global__ void k_taylor_block(int norb, const double* __restrict__ y, const double* __restrict__ P2,
                               const double* __restrict__ P3, const double* __restrict__ P4,
                               TaylorBlock tb, const ExpmScratch* __restrict__ sc,
                               double* __restrict__ out, long long yinst, long long ab) {
  const long long inst = blockIdx.y;
  const long long n2 = (long long)norb * norb;
  const double s = sc[inst].scale;
  const double w1 = tb.c[1] * s, w2 = tb.c[2] * (s * s), w3 = tb.c[3] * (s * s * s);
  const double w4 = tb.np > 4 ? tb.c[4] * ((s * s) * (s * s)) : 0.0;
  y += inst * yinst;
  P2 += inst * ab;
  P3 += inst * ab;
  P4 += inst * ab;
  out += inst * ab;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / norb), q = (int)(i - (long long)r * norb);
    double v = (r == q ? tb.c[0] : 0.0) + w1 * y[i] + w2 * P2[i] + w3 * P3[i];
    if (tb.np > 4) v += w4 * P4[i];
    out[i] = v;
  }
}

// U_i = buffer holding instance i's result after s_i squarings (ping-pong
// parity); A and B at instance stride ab, U at norb^2.
__global__ void k_select(int norb, const double* __restrict__ A, const double* __restrict__ B,
                         long long ab, const ExpmScratch* __restrict__ sc, double* __restrict__ U) {
  const long long n2 = (long long)norb * norb;
  const long long y = blockIdx.y;
  const double* src = ((sc[y].s & 1) ? B : A) + y * ab;
  U += y * n2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x)
    U[i] = src[i];
}

__global__ void k_adam(long long n2, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, double b1, double b2, double c1, double c2,
                       double lr, double eps, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const double mh = mi / c1, vh = vi / c2;
    y[i] = -lr * mh / (sqrt(vh) + eps);
  }
}

// Orthonormality check of the orbitals: err = max|E| of E = C^T S C - I
// (a non-finite entry counts as +inf), sc->s = (err > tol), sc->scale = err,
// *err_out = err when given, and M = I - E/2 for the repair step.
__global__ __launch_bounds__(1024) void k_orth_check(int norb, const double* __restrict__ E,
                                                     double tol, double* __restrict__ M,
                                                     ExpmScratch* __restrict__ sc,
                                                     double* __restrict__ err_out) {
  __shared__ double red[1024];
  const long long n2 = (long long)norb * norb;
  double m = 0.0;
  for (long long i = threadIdx.x; i < n2; i += 1024) {
    const double e = E[i];
    const double a = fabs(e);
    m = a <= 1.7976931348623157e308 ? fmax(m, a) : INFINITY;
    const long long p = i / norb, q = i - p * norb;
    M[i] = (p == q ? 1.0 : 0.0) - 0.5 * e;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sc->s = red[0] > tol ? 1 : 0;
    sc->pad = 0;
    sc->scale = red[0];
    if (err_out) *err_out = red[0];
  }
}

inline int grid_for(long long n, int thr) {
  long long g = (n + thr - 1) / thr;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

// Split-K plan for the small products of this file: 128-wide tiles once
// there are 64 of them (Norb >= ~1000), else 64-wide tiles, and enough splits
// of K for about 384 (128-wide) or 256 (64-wide) workgroups.  At Norb = 500
// the 64-wide plan (4 splits) takes exp(y) from 0.56 to 0.35 ms against 128-wide
// tiles with 24 splits, whose partials (2 MB each) dominate; at Norb = 1000 the
// 128-wide plan is faster (1.14 vs 1.28 ms).
struct SplitPlan {
  int tile, ns;
};
SplitPlan split_for(int rows, int cols, int K) {
  const int t128 = ((rows + 127) / 128) * ((cols + 127) / 128);
  const int tile = t128 >= 64 ? 128 : 64;
  const int tiles = tile == 128 ? t128 : ((rows + 63) / 64) * ((cols + 63) / 64);
  const int target = tile == 128 ? 384 : 256;
  int ns = (target + tiles - 1) / tiles;
  const int maxs = (K + 15) / 16;          // at least one 16-deep stage per split
  if (ns > maxs) ns = maxs;
  if (ns > 32) ns = 32;
  if (ns < 1) ns = 1;
  return {tile, ns};
}

// part_i[c] = sum over k in split c of X_i(k, m) Y_i(k, n) for instances
// i < ninst (X_i = X + i*xinst, Y_i = Y + i*yinst, part_i = part + i*nsplit*M*N);
// X given k-major or m-major.  With pred_sc, instance i runs only when
// pred_sc[i].s > pred_gt.
int gemm_split(int ninst, int M, int N, int K, const double* X, bool x_kmajor, long long ldx,
               long long xinst, const double* Y, long long ldy, long long yinst, double* part,
               SplitPlan plan, const ExpmScratch* pred_sc, int pred_gt, hipStream_t st) {
  const int nsplit = plan.ns;
  const int kc = (K + nsplit - 1) / nsplit;
  GemmDesc g{};
  g.M = M; g.N = N; g.K = kc; g.Ktot = K;
  g.tile = plan.tile;
  g.batch = ninst * nsplit; g.binner = nsplit; g.fold = 1;
  g.X = X; g.ldx = ldx; g.sx = x_kmajor ? (long long)kc * ldx : (long long)kc; g.x_kmajor = x_kmajor;
  g.sx2 = xinst;
  g.Y = Y; g.ldy = ldy; g.sy = (long long)kc * ldy; g.sy2 = yinst;
  g.Out = part; g.ldo = N; g.so = (long long)M * N; g.so2 = (long long)nsplit * M * N;
  if (pred_sc) {
    g.pred = &pred_sc->s;
    g.pred_so = (long long)(sizeof(ExpmScratch) / sizeof(int));
    g.pred_gt = pred_gt;
  }
  return gemm_tn(g, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
}

int combine(int ninst, int rows, int cols, const double* part, int nparts, double diag_c,
            double coef_mul, const ExpmScratch* sc, const ExpmScratch* pred_sc, int pred_gt,
            double* out, long long oinst, hipStream_t st) {
  const long long n = (long long)rows * cols;
  hipLaunchKernelGGL(k_combine, dim3(grid_for(n, 256), ninst), dim3(256), 0, st, rows, cols, part,
                     nparts, n, diag_c, coef_mul, sc, pred_sc, pred_gt, out, (long long)nparts * n,
                     oinst);
  return launch_status();
}

}  // namespace

// Workspace of ninst simultaneous exponentials: scaling records, A and B
// ping-pong buffers and split partials per instance.
size_t expm_ws(int norb, int ninst) {
  const size_t n2 = align256((size_t)norb * norb * sizeof(double));
  const int ns = split_for(norb, norb, norb).ns;
  // A, B (ping-pong), the powers y^2, y^3, y^4, split partials
  return align256((size_t)ninst * sizeof(ExpmScratch)) + (size_t)ninst * (5 * n2 + (size_t)ns * n2);
}

size_t rotate_ws(int nbf, int norb, int ninst) {
  const int ns = split_for(nbf, norb, norb).ns;
  return (size_t)ninst * ns * align256((size_t)nbf * norb * sizeof(double));
}

// Cout_i = C_i U_i for i < ninst (C, Cout stride nbf*norb, U stride norb^2).
int rotate_orbitals(int nbf, int norb, const double* C, const double* U, double* Cout, void* ws,
                    hipStream_t st, int ninst) {
  const SplitPlan plan = split_for(nbf, norb, norb);
  double* part = (double*)ws;
  const long long cs = (long long)nbf * norb, n2 = (long long)norb * norb;
  // Cout[mu][p] = sum_q C[mu][q] U[q][p]: X(k=q, m=mu) = C[mu][q] (m-major)
  int rc = gemm_split(ninst, nbf, norb, norb, C, false, norb, cs, U, norb, n2, part, plan, nullptr, 0,
                      st);
  if (rc != NOF_OK) return rc;
  return combine(ninst, nbf, norb, part, plan.ns, 0.0, 1.0, nullptr, nullptr, 0, Cout, cs, st);
}

// U_i = exp(y_i) for i < ninst (y, U stride norb^2); each instance takes its
// own scaling power, so its result does not depend on the other instances.
int expm_antisym(int norb, const double* y, double* U, void* ws, hipStream_t st, int ninst) {
  char* w = (char*)ws;
  ExpmScratch* sc = (ExpmScratch*)w;
  const size_t n2b = align256((size_t)norb * norb * sizeof(double));
  const long long n2 = (long long)norb * norb;
  const long long ab = (long long)(n2b / sizeof(double));   // instance stride of A and B
  double* A = (double*)(w + align256((size_t)ninst * sizeof(ExpmScratch)));
  double* Bm = A + (long long)ninst * ab;
  double* P2 = Bm + (long long)ninst * ab;
  double* P3 = P2 + (long long)ninst * ab;
  double* P4 = P3 + (long long)ninst * ab;
  double* part = P4 + (long long)ninst * ab;
  const SplitPlan plan = split_for(norb, norb, norb);
  const int ns = plan.ns;
  const dim3 eg(grid_for(n2, 256), ninst);
  hipLaunchKernelGGL(k_norm_scale, dim3(ninst), dim3(1024), 0, st, norb, y, sc);
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  // unscaled powers: P = X Y with X(k, m) = X[m][k] (m-major)
  auto power = [&](const double* X, long long xinst, const double* Y, long long yinst, double* out) {
    int r = gemm_split(ninst, norb, norb, norb, X, false, norb, xinst, Y, norb, yinst, part, plan,
                       nullptr, 0, st);
    if (r != NOF_OK) return r;
    return combine(ninst, norb, norb, part, ns, 0.0, 1.0, nullptr, nullptr, 0, out, ab, st);
  };
  if ((rc = power(y, n2, y, n2, P2)) != NOF_OK) return rc;      // y^2
  if ((rc = power(P2, ab, y, n2, P3)) != NOF_OK) return rc;     // y^3
  if ((rc = power(P2, ab, P2, ab, P4)) != NOF_OK) return rc;    // y^4
  // Taylor coefficients 1/k!, k = 0 .. 12, in blocks of four (the last holds five)
  double f[kTaylor + 1];
  f[0] = 1.0;
  for (int k = 1; k <= kTaylor; ++k) f[k] = f[k - 1] / k;
  auto block = [&](int j, double* out) {
    TaylorBlock tb{};
    tb.np = j == 2 ? 5 : 4;
    for (int i = 0; i < tb.np; ++i) tb.c[i] = f[4 * j + i];
    hipLaunchKernelGGL(k_taylor_block, eg, dim3(256), 0, st, norb, y, P2, P3, P4, tb, sc, out, n2, ab);
    return launch_status();
  };
  // A = B2;  A = B1 + x^4 A;  A = B0 + x^4 A
  if ((rc = block(2, A)) != NOF_OK) return rc;
  for (int j = 1; j >= 0; --j) {
    if ((rc = block(j, Bm)) != NOF_OK) return rc;
    rc = gemm_split(ninst, norb, norb, norb, P4, false, norb, ab, A, norb, ab, part, plan, nullptr, 0, st);
    if (rc != NOF_OK) return rc;
    hipLaunchKernelGGL(k_combine_x4, eg, dim3(256), 0, st, n2, part, ns, n2, sc, Bm, A,
                       (long long)ns * n2, ab);
    if ((rc = launch_status()) != NOF_OK) return rc;
  }
  // squarings i = 0 .. s-1, ping-pong A -> B -> A ... (instances with s <= i skip)
  double* cur = A;
  double* nxt = Bm;
  for (int i = 0; i < kMaxSquare; ++i) {
    // nxt = cur cur: X(k, m) = cur[m][k] (m-major)
    rc = gemm_split(ninst, norb, norb, norb, cur, false, norb, ab, cur, norb, ab, part, plan, sc, i, st);
    if (rc != NOF_OK) return rc;
    rc = combine(ninst, norb, norb, part, ns, 0.0, 1.0, nullptr, sc, i, nxt, ab, st);
    if (rc != NOF_OK) return rc;
    double* t = cur; cur = nxt; nxt = t;
  }
  hipLaunchKernelGGL(k_select, dim3(grid_for(n2, 256), ninst), dim3(256), 0, st, norb, A, Bm, ab, sc,
                     U);
  return launch_status();
}

// Workspace of orthonormalize: check record, E, M, S C, split partials.
size_t orth_ws(int nbf, int norb) {
  const size_t n2b = align256((size_t)norb * norb * sizeof(double));
  const size_t cb = align256((size_t)nbf * norb * sizeof(double));
  const size_t ng = (size_t)split_for(norb, norb, nbf).ns * n2b;
  const size_t nc = (size_t)std::max(split_for(nbf, norb, norb).ns, split_for(nbf, norb, nbf).ns) * cb;
  return 256 + 2 * n2b + cb + std::max(ng, nc);
}

// C <- C (I - E/2) when max|E| > tol, E = C^T S C - I (S NULL: identity);
// *err (device, may be NULL) = max|E| before the repair.  Nothing is read
// back: the repair launches are predicated on the check record.
int orthonormalize(int nbf, int norb, double* C, const double* S, double tol, double* err, void* ws,
                   hipStream_t st) {
  char* w = (char*)ws;
  const size_t n2b = align256((size_t)norb * norb * sizeof(double));
  const size_t cb = align256((size_t)nbf * norb * sizeof(double));
  ExpmScratch* sc = (ExpmScratch*)w;
  double* E = (double*)(w + 256);
  double* M = (double*)(w + 256 + n2b);
  double* SC = (double*)(w + 256 + 2 * n2b);
  double* part = (double*)(w + 256 + 2 * n2b + cb);
  int rc;
  const double* Y = C;
  if (S) {
    // SC[mu][p] = sum_nu S[mu][nu] C[nu][p]: X(k=nu, m=mu) = S[mu][nu] (m-major)
    const SplitPlan ps = split_for(nbf, norb, nbf);
    if ((rc = gemm_split(1, nbf, norb, nbf, S, false, nbf, 0, C, norb, 0, part, ps, nullptr, 0, st)) !=
        NOF_OK)
      return rc;
    if ((rc = combine(1, nbf, norb, part, ps.ns, 0.0, 1.0, nullptr, nullptr, 0, SC, 0, st)) != NOF_OK)
      return rc;
    Y = SC;
  }
  // E[p][q] = sum_mu C[mu][p] Y[mu][q] - delta_pq: X(k=mu, m=p) = C[mu][p] (k-major)
  const SplitPlan pg = split_for(norb, norb, nbf);
  if ((rc = gemm_split(1, norb, norb, nbf, C, true, norb, 0, Y, norb, 0, part, pg, nullptr, 0, st)) !=
      NOF_OK)
    return rc;
  if ((rc = combine(1, norb, norb, part, pg.ns, -1.0, 1.0, nullptr, nullptr, 0, E, 0, st)) != NOF_OK)
    return rc;
  hipLaunchKernelGGL(k_orth_check, dim3(1), dim3(1024), 0, st, norb, E, tol, M, sc, err);
  if ((rc = launch_status()) != NOF_OK) return rc;
  // C <- C M, both launches predicated on sc->s: X(k=q, m=mu) = C[mu][q] (m-major)
  const SplitPlan pc = split_for(nbf, norb, norb);
  if ((rc = gemm_split(1, nbf, norb, norb, C, false, norb, 0, M, norb, 0, part, pc, sc, 0, st)) != NOF_OK)
    return rc;
  return combine(1, nbf, norb, part, pc.ns, 0.0, 1.0, nullptr, sc, 0, C, 0, st);
}

int adam_step(int norb, const double* g, double* m, double* v, int t, double lr, double beta1,
              double beta2, double eps, double* y, hipStream_t st) {
  const long long n2 = (long long)norb * norb;
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n2, 256)), dim3(256), 0, st, n2, g, m, v, beta1, beta2,
                     c1, c2, lr, eps, y);
  return launch_status();
}

}  // namespace nof
