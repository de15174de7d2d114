// Learned warm start of the occupation optimiser: per-orbital features, a
// 5 -> 128 -> 128 -> 1 perceptron (tanh hidden units, output angle
// theta = (pi/2) sigmoid(z), n = cos^2 theta) and its training (MSE on theta,
// ADAM), all in FP32 with FP64 reductions.
//
// Parameters are one flat FP32 vector: W1 [5][128], b1 [128], W2 [128][128],
// b2 [128], w3 [128], b3.
//
// Forward and backward run fused per block of 64 rows: W2 is staged once per
// block in LDS with rows padded to 129 floats (so both W2[k][j] over j and
// W2[k][j] over k are conflict-free), the hidden activations of the block stay
// in LDS, and each block writes its partial gradient; a second kernel sums the
// partials in a fixed order (bitwise-repeatable training).
#include <math.h>

#include "common.h"

namespace nof {
namespace {

constexpr int DI = 5, DH = 128;
constexpr int O_W1 = 0, O_B1 = O_W1 + DI * DH, O_W2 = O_B1 + DH, O_B2 = O_W2 + DH * DH,
              O_W3 = O_B2 + DH, O_B3 = O_W3 + DH, NP = O_B3 + 1;
constexpr int RB = 64;            // rows per block
constexpr int MT = 256;           // threads per block
constexpr int HP = DH + 1;        // padded LDS row
constexpr double kHalfPi = 1.5707963267948966;

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

template <bool TRAIN>
__global__ __launch_bounds__(MT) void k_mlp(int rows, const float* __restrict__ X,
                                            const float* __restrict__ P,
                                            const float* __restrict__ target,
                                            float* __restrict__ theta,
                                            float* __restrict__ gpart,
                                            double* __restrict__ lpart) {
  __shared__ float W2s[DH][HP];
  __shared__ float H1[RB][HP];
  __shared__ float H2[RB][HP];
  __shared__ float Xs[RB][DI];
  __shared__ float dz[RB];
  __shared__ double lred[RB];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * RB;
  const int nr = min(RB, rows - r0);
  for (int e = tid; e < DH * DH; e += MT) W2s[e / DH][e % DH] = P[O_W2 + e];
  for (int e = tid; e < RB * DI; e += MT) {
    const int r = e / DI, k = e % DI;
    Xs[r][k] = r < nr ? X[(long long)(r0 + r) * DI + k] : 0.f;
  }
  __syncthreads();
  const int j = tid & (DH - 1);
  const int rh = tid >> 7;                       // 0 or 1: rows rh, rh+2, ...
  // layer 1
  {
    float w[DI];
#pragma unroll
    for (int k = 0; k < DI; ++k) w[k] = P[O_W1 + k * DH + j];
    const float bj = P[O_B1 + j];
    for (int i = 0; i < RB / 2; ++i) {
      const int r = rh + 2 * i;
      float a = bj;
#pragma unroll
      for (int k = 0; k < DI; ++k) a = fmaf(Xs[r][k], w[k], a);
      H1[r][j] = tanhf(a);
    }
  }
  __syncthreads();
  // layer 2: H2[r][j] = tanh(sum_k H1[r][k] W2[k][j] + b2[j])
  {
    float acc[RB / 2];
    const float bj = P[O_B2 + j];
#pragma unroll
    for (int i = 0; i < RB / 2; ++i) acc[i] = bj;
    for (int k = 0; k < DH; ++k) {
      const float wk = W2s[k][j];
#pragma unroll
      for (int i = 0; i < RB / 2; ++i) acc[i] = fmaf(H1[rh + 2 * i][k], wk, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < RB / 2; ++i) H2[rh + 2 * i][j] = tanhf(acc[i]);
  }
  __syncthreads();
  // layer 3: one wave per 16 rows
  {
    const int lane = tid & 63, wv = tid >> 6;
    const float w3a = P[O_W3 + lane], w3b = P[O_W3 + 64 + lane];
    const float b3 = P[O_B3];
    for (int i = 0; i < RB / 4; ++i) {
      const int r = wv * (RB / 4) + i;
      float s = H2[r][lane] * w3a + H2[r][64 + lane] * w3b;
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0) {
        const float sg = sigm(s + b3);
        const float th = (float)kHalfPi * sg;
        if (r < nr) {
          if (!TRAIN) theta[r0 + r] = th;
          if (TRAIN) {
            const float res = th - target[r0 + r];
            dz[r] = 2.0f * res / (float)rows * (float)kHalfPi * sg * (1.0f - sg);
            lred[r] = (double)res * (double)res;
          }
        } else if (TRAIN) {
          dz[r] = 0.f;
          lred[r] = 0.0;
        }
      }
    }
  }
  if (!TRAIN) return;
  __syncthreads();
  float* G = gpart + (long long)blockIdx.x * NP;
  // loss partial, dw3, db3
  if (tid == 0) {
    double s = 0.0;
    for (int r = 0; r < RB; ++r) s += lred[r];
    lpart[blockIdx.x] = s;
    float d3 = 0.f;
    for (int r = 0; r < RB; ++r) d3 += dz[r];
    G[O_B3] = d3;
  }
  if (tid < DH) {
    float s = 0.f;
    for (int r = 0; r < RB; ++r) s = fmaf(H2[r][tid], dz[r], s);
    G[O_W3 + tid] = s;
  }
  __syncthreads();
  // dA2 = dz w3 (1 - H2^2), stored over H2
  {
    const float w3j = P[O_W3 + j];
    for (int i = 0; i < RB / 2; ++i) {
      const int r = rh + 2 * i;
      const float h = H2[r][j];
      H2[r][j] = dz[r] * w3j * (1.0f - h * h);
    }
  }
  __syncthreads();
  // dW2[k][j] = sum_r H1[r][k] dA2[r][j]; db2[j] = sum_r dA2[r][j]
  {
    for (int kk = 0; kk < DH / 2; ++kk) {
      const int k = rh + 2 * kk;
      float s = 0.f;
      for (int r = 0; r < RB; ++r) s = fmaf(H1[r][k], H2[r][j], s);
      G[O_W2 + k * DH + j] = s;
    }
    if (tid < DH) {
      float s = 0.f;
      for (int r = 0; r < RB; ++r) s += H2[r][tid];
      G[O_B2 + tid] = s;
    }
  }
  // dH1[r][k] = sum_j dA2[r][j] W2[k][j]; thread owns k = j (column index reused)
  float dh[RB / 2];
  {
    const int k = j;
#pragma unroll
    for (int i = 0; i < RB / 2; ++i) dh[i] = 0.f;
    for (int jj = 0; jj < DH; ++jj) {
      const float w = W2s[k][jj];
#pragma unroll
      for (int i = 0; i < RB / 2; ++i) dh[i] = fmaf(H2[rh + 2 * i][jj], w, dh[i]);
    }
  }
  __syncthreads();                                // all reads of H1 for dW2 are done
  for (int i = 0; i < RB / 2; ++i) {
    const int r = rh + 2 * i;
    const float h = H1[r][j];
    H1[r][j] = dh[i] * (1.0f - h * h);            // dA1
  }
  __syncthreads();
  // dW1[k][j] = sum_r X[r][k] dA1[r][j]; db1[j]
  if (tid < DH) {
    float s1[DI] = {0, 0, 0, 0, 0};
    float sb = 0.f;
    for (int r = 0; r < RB; ++r) {
      const float a = H1[r][tid];
      sb += a;
#pragma unroll
      for (int k = 0; k < DI; ++k) s1[k] = fmaf(Xs[r][k], a, s1[k]);
    }
#pragma unroll
    for (int k = 0; k < DI; ++k) G[O_W1 + k * DH + tid] = s1[k];
    G[O_B1 + tid] = sb;
  }
}

__global__ void k_mlp_reduce(int nblk, const float* __restrict__ gpart,
                             const double* __restrict__ lpart, float* __restrict__ grad,
                             float* __restrict__ loss, int rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NP) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += (double)gpart[(long long)b * NP + i];
    grad[i] = (float)s;
  }
  if (i == NP && loss) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += lpart[b];
    *loss = (float)(s / rows);
  }
}

__global__ void k_mlp_adam(int n, float* __restrict__ p, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, float b1, float b2,
                           float c1, float c2, float lr, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Raw features of orbital r, then per-feature z-scores over the instance.
__global__ __launch_bounds__(1024) void k_mlp_features(int norb, const double* __restrict__ hdiag,
                                                       int hstride, const double* __restrict__ J,
                                                       const double* __restrict__ K,
                                                       double* __restrict__ F,
                                                       float* __restrict__ X) {
  __shared__ double red[1024];
  __shared__ double mu[DI], sd[DI];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int r = wv; r < norb; r += 16) {
    double sj = 0.0, sk = 0.0;
    for (int q = lane; q < norb; q += 64) {
      sj += J[(long long)r * norb + q];
      sk += K[(long long)r * norb + q];
    }
    for (int o = 32; o > 0; o >>= 1) {
      sj += __shfl_xor(sj, o, 64);
      sk += __shfl_xor(sk, o, 64);
    }
    if (lane == 0) {
      F[(long long)r * DI + 0] = J[(long long)r * norb + r];
      F[(long long)r * DI + 1] = K[(long long)r * norb + r];
      F[(long long)r * DI + 2] = hdiag[(long long)r * hstride];
      F[(long long)r * DI + 3] = sj / norb;
      F[(long long)r * DI + 4] = sk / norb;
    }
  }
  __syncthreads();
  for (int k = 0; k < DI; ++k) {
    double s = 0.0;
    for (int r = tid; r < norb; r += 1024) s += F[(long long)r * DI + k];
    red[tid] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double m = red[0] / norb;
    __syncthreads();
    double s2 = 0.0;
    for (int r = tid; r < norb; r += 1024) {
      const double dv = F[(long long)r * DI + k] - m;
      s2 += dv * dv;
    }
    red[tid] = s2;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      mu[k] = m;
      const double s = sqrt(red[0] / norb);
      sd[k] = s > 0.0 ? s : 1.0;
    }
    __syncthreads();
  }
  for (int e = tid; e < norb * DI; e += 1024) {
    const int k = e % DI;
    X[e] = (float)((F[e] - mu[k]) / sd[k]);
  }
}

// Warm start: n = cos^2 theta, projected per subspace onto the sum rule
// (and n_g >= 1/2 for the trigonometric map), then the inverse mapping.
__global__ void k_warm_gamma(int norb, int ns, int ng, const int* __restrict__ members, int map,
                             const float* __restrict__ theta, double nfloor,
                             double* __restrict__ gamma, int* __restrict__ info) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ns) return;
  const int* row = members + (long long)g * (ng + 1);
  double vals[65];
  if (ng + 1 > 65) { if (info) info[2] = NOF_E_DIM; return; }
  double tot = 0.0;
  for (int i = 0; i <= ng; ++i) {
    const int q = row[i];
    if (q < 0 || q >= norb) { if (info) info[2] = NOF_E_ARG; return; }
    const double c = cos((double)theta[q]);
    vals[i] = c * c;
    tot += vals[i];
  }
  double s2 = 0.0;
  for (int i = 0; i <= ng; ++i) {
    double v = tot > 0.0 ? vals[i] / tot : 1.0 / (ng + 1);
    vals[i] = v < nfloor ? nfloor : v;
  }
  if (map == NOF_MAP_TRIG && vals[0] < 0.5) {
    double rest = 0.0;
    for (int i = 1; i <= ng; ++i) rest += vals[i];
    for (int i = 1; i <= ng; ++i) vals[i] *= 0.5 / rest;
    vals[0] = 0.5;
  }
  for (int i = 0; i <= ng; ++i) s2 += vals[i];
  for (int i = 0; i <= ng; ++i) vals[i] /= s2;
  double* out = gamma + (long long)g * ng;
  if (map == NOF_MAP_SOFTMAX) {
    for (int i = 0; i < ng; ++i) out[i] = log(vals[1 + i] / vals[0]);
    return;
  }
  // inverse trigonometric map
  double t = 2.0 * vals[0] - 1.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  out[0] = acos(sqrt(t));
  double rem = 1.0 - vals[0];
  for (int i = 1; i < ng; ++i) {
    double f = rem > 0.0 ? vals[i] / rem : 0.0;
    f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    out[i] = asin(sqrt(f));
    rem -= vals[i];
  }
}

__global__ void k_targets(int n, const double* __restrict__ occ, float* __restrict__ theta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = occ[i];
  v = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
  theta[i] = (float)acos(sqrt(v));
}

}  // namespace

int mlp_targets(int n, const double* occ, float* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_targets, dim3((n + 255) / 256), dim3(256), 0, st, n, occ, theta);
  return launch_status();
}

int mlp_nparams() { return NP; }

size_t mlp_ws(int rows) {
  const size_t nblk = (size_t)(rows + RB - 1) / RB;
  return align256(nblk * NP * sizeof(float)) + align256(nblk * sizeof(double));
}

int mlp_forward(int rows, const float* X, const float* P, float* theta, hipStream_t st) {
  const int nblk = (rows + RB - 1) / RB;
  hipLaunchKernelGGL((k_mlp<false>), dim3(nblk), dim3(MT), 0, st, rows, X, P, nullptr, theta,
                     nullptr, nullptr);
  return launch_status();
}

int mlp_loss_grad(int rows, const float* X, const float* target, const float* P, float* grad,
                  float* loss, void* ws, hipStream_t st) {
  const int nblk = (rows + RB - 1) / RB;
  float* gpart = (float*)ws;
  double* lpart = (double*)((char*)ws + align256((size_t)nblk * NP * sizeof(float)));
  hipLaunchKernelGGL((k_mlp<true>), dim3(nblk), dim3(MT), 0, st, rows, X, P, target, nullptr,
                     gpart, lpart);
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, nblk, gpart,
                     lpart, grad, loss, rows);
  return launch_status();
}

int mlp_adam(int n, float* p, const float* g, float* m, float* v, int t, float lr, float b1,
             float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((n + 255) / 256), dim3(256), 0, st, n, p, g, m, v, b1, b2,
                     c1, c2, lr, eps);
  return launch_status();
}

int mlp_features(int norb, const double* hdiag, int hstride, const double* J, const double* K,
                 float* X, void* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_features, dim3(1), dim3(1024), 0, st, norb, hdiag, hstride, J, K,
                     (double*)ws, X);
  return launch_status();
}

int mlp_warm_gamma(int norb, int ns, int ng, const int* members, int map, const float* theta,
                   double nfloor, double* gamma, int* info, hipStream_t st) {
  hipLaunchKernelGGL(k_warm_gamma, dim3((ns + 127) / 128), dim3(128), 0, st, norb, ns, ng,
                     members, map, theta, nfloor, gamma, info);
  return launch_status();
}

}  // namespace nof
