// FP64 orbital-rotation step (NO Optimization: U = exp(y) with y
// antisymmetric, C <- C U, and the ADAM update of y from the orbital gradient).
//
// exp(y) is evaluated by scaling and squaring with a degree-12 Taylor
// polynomial (Higham, "The scaling and squaring method for the matrix
// exponential revisited", SIAM J. Matrix Anal. Appl. 26 (2005)): the scaling
// power s is chosen on the device from ||y||_1 so that ||y / 2^s||_1 <= 1/4,
// where the truncation error is below 3e-18; the polynomial is applied in
// Horner form and then squared s times.  Nothing is read back to the host,
// so the whole step stays asynchronous (and graph capturable): the squaring
// launches beyond s exit immediately.
#include <math.h>

#include "common.h"

namespace nof {
namespace {

constexpr int kTaylor = 12;
constexpr int kMaxSquare = 16;      // ||y||_1 up to 2^16 / 4
constexpr double kTheta = 0.25;

struct ExpmScratch {
  int s;
  int pad;
  double scale;   // 2^-s
};

__global__ __launch_bounds__(1024) void k_norm1(int norb, const double* __restrict__ y,
                                                ExpmScratch* __restrict__ sc) {
  __shared__ double red[1024];
  double mx = 0.0;
  for (int j = threadIdx.x; j < norb; j += 1024) {
    double c = 0.0;
    for (int i = 0; i < norb; ++i) c += fabs(y[(long long)i * norb + j]);
    mx = fmax(mx, c);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nrm = red[0];
    int s = 0;
    double sc_ = 1.0;
    while (nrm * sc_ > kTheta && s < kMaxSquare) { ++s; sc_ *= 0.5; }
    sc->s = s;
    sc->scale = sc_;
  }
}

__global__ void k_identity(int norb, double* __restrict__ R) {
  const long long n2 = (long long)norb * norb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / norb), c = (int)(i - (long long)r * norb);
    R[i] = r == c ? 1.0 : 0.0;
  }
}

// R = I - (2^-s / k) * Tm, where Tm = y^T R_prev = -(y R_prev)
__global__ void k_horner(int norb, const double* __restrict__ Tm, double k,
                         const ExpmScratch* __restrict__ sc, double* __restrict__ R) {
  const double a = sc->scale / k;
  const long long n2 = (long long)norb * norb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / norb), c = (int)(i - (long long)r * norb);
    R[i] = (r == c ? 1.0 : 0.0) - a * Tm[i];
  }
}

// U = buffer holding the result after s squarings (ping-pong parity)
__global__ void k_select(int norb, const double* __restrict__ A, const double* __restrict__ B,
                         const ExpmScratch* __restrict__ sc, double* __restrict__ U) {
  const double* src = (sc->s & 1) ? B : A;
  const long long n2 = (long long)norb * norb;
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

inline int grid_for(long long n, int thr) {
  long long g = (n + thr - 1) / thr;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

GemmDesc square_desc(int norb, const double* Rin, double* Rout) {
  // Rout = Rin Rin: X(k,m) = Rin[m][k] (row-major Rin read as [m][k])
  GemmDesc g{};
  g.M = norb; g.N = norb; g.K = norb; g.Ktot = 0;
  g.batch = 1; g.fold = 1;
  g.X = Rin; g.ldx = norb; g.sx = 0; g.x_kmajor = false;
  g.Y = Rin; g.ldy = norb; g.sy = 0;
  g.Out = Rout; g.ldo = norb; g.so = 0;
  return g;
}

}  // namespace

size_t expm_ws(int norb) {
  const size_t n2 = (size_t)norb * norb * sizeof(double);
  return align256(sizeof(ExpmScratch)) + 3 * align256(n2);
}

int expm_antisym(int norb, const double* y, double* U, void* ws, hipStream_t st) {
  char* w = (char*)ws;
  ExpmScratch* sc = (ExpmScratch*)w;
  const size_t n2b = align256((size_t)norb * norb * sizeof(double));
  double* A = (double*)(w + align256(sizeof(ExpmScratch)));
  double* Bm = (double*)((char*)A + n2b);
  double* Tm = (double*)((char*)Bm + n2b);
  const long long n2 = (long long)norb * norb;
  const int gr = grid_for(n2, 256);
  hipLaunchKernelGGL(k_norm1, dim3(1), dim3(1024), 0, st, norb, y, sc);
  hipLaunchKernelGGL(k_identity, dim3(gr), dim3(256), 0, st, norb, A);
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  // Horner: R <- I + (x/k) R for k = 12..1, x = y / 2^s
  for (int k = kTaylor; k >= 1; --k) {
    GemmDesc g{};
    g.M = norb; g.N = norb; g.K = norb; g.Ktot = 0;
    g.batch = 1; g.fold = 1;
    g.X = y; g.ldx = norb; g.sx = 0; g.x_kmajor = true;     // y^T R
    g.Y = A; g.ldy = norb; g.sy = 0;
    g.Out = Tm; g.ldo = norb; g.so = 0;
    rc = gemm_tn(g, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
    if (rc != NOF_OK) return rc;
    hipLaunchKernelGGL(k_horner, dim3(gr), dim3(256), 0, st, norb, Tm, (double)k, sc, A);
    rc = launch_status();
    if (rc != NOF_OK) return rc;
  }
  // squarings i = 0 .. s-1, ping-pong A -> B -> A ...
  double* cur = A;
  double* nxt = Bm;
  for (int i = 0; i < kMaxSquare; ++i) {
    GemmDesc g = square_desc(norb, cur, nxt);
    g.pred = &sc->s;
    g.pred_gt = i;
    rc = gemm_tn(g, NOF_F64, NOF_F64, NOF_F64, NOF_P_F64, st);
    if (rc != NOF_OK) return rc;
    double* t = cur; cur = nxt; nxt = t;
  }
  hipLaunchKernelGGL(k_select, dim3(gr), dim3(256), 0, st, norb, A, Bm, sc, U);
  return launch_status();
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
