// Finite-field NLOP step (NLOPs: Polarizabilities and Hyperpolarizabilities):
// the electronic dipole of a NOF state and the Romberg-Richardson refinement
// of the centred-difference polarizability and hyperpolarizabilities.
#include <cmath>

#include "common.h"

namespace nof {
namespace {

constexpr int MAXPT = 16;

// mu = -2 sum_p n_p X_pp, X = C^T d C; one workgroup, fixed-order tree.
__global__ void k_dipole(int norb, const double* __restrict__ X, const double* __restrict__ n,
                         double* __restrict__ mu) {
  __shared__ double red[256];
  double s = 0.0;
  for (int p = threadIdx.x; p < norb; p += blockDim.x) s += n[p] * X[(long long)p * norb + p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mu = -2.0 * red[0];
}

// Centred estimate of property prop (0 alpha, 1 beta, 2 gamma) at step h.
__device__ double estimate(int prop, double mu0, double mp, double mm, double m2p, double m2m, double h) {
  if (prop == 0) return (mp - mm) / (2.0 * h);
  if (prop == 1) return (mp - 2.0 * mu0 + mm) / (h * h);
  return (m2p - 2.0 * mp + 2.0 * mm - m2m) / (2.0 * h * h * h);
}

// One thread per property: the Romberg triangle (p = 2) over the dyadic
// ladder and the selection of the smallest vertical difference (its value
// taken from the next column; equal differences: smallest magnitude).
// table[prop][k][j] (npoint x npoint, NaN outside the triangle);
// result[prop] = (value, uncertainty, k, j).
__global__ void k_nlop(int npoint, double step, const double* __restrict__ mu0p,
                       const double* __restrict__ mu_p, const double* __restrict__ mu_m,
                       double* __restrict__ table, double* __restrict__ result) {
  const int prop = threadIdx.x;
  if (prop >= 3) return;
  double R[MAXPT][MAXPT];
  const double mu0 = *mu0p;
  double h = step;
  for (int k = 0; k < npoint; ++k, h *= 2.0)
    R[k][0] = estimate(prop, mu0, mu_p[k], mu_m[k], mu_p[k + 1], mu_m[k + 1], h);
  double f = 1.0;
  for (int j = 1; j < npoint; ++j) {
    f *= 4.0;
    for (int k = 0; k < npoint - j; ++k) R[k][j] = R[k][j - 1] + (R[k][j - 1] - R[k + 1][j - 1]) / (f - 1.0);
  }
  double* T = table + (long long)prop * npoint * npoint;
  for (int k = 0; k < npoint; ++k)
    for (int j = 0; j < npoint; ++j) T[k * npoint + j] = (k + j < npoint) ? R[k][j] : NAN;
  double bd = INFINITY, bv = NAN;
  int bk = -1, bj = -1;
  for (int j = 0; j + 1 < npoint; ++j)
    for (int k = 0; k + j + 1 < npoint; ++k) {
      const double dl = fabs(R[k + 1][j] - R[k][j]);
      const double cand = R[k][j + 1];
      if (dl < bd || (dl == bd && fabs(cand) < fabs(bv))) {
        bd = dl; bv = cand; bk = k; bj = j;
      }
    }
  if (npoint == 1) { bv = R[0][0]; bd = NAN; bk = 0; bj = 0; }
  result[prop * 4 + 0] = bv;
  result[prop * 4 + 1] = bd;
  result[prop * 4 + 2] = bk;
  result[prop * 4 + 3] = bj;
}

// Isotropic polarizability and anisotropy (Raman convention) of the diagonal
// components a[0..2]: out = ((a0 + a1 + a2)/3, sqrt(((a0-a1)^2 + (a1-a2)^2 + (a2-a0)^2)/2)).
__global__ void k_iso(const double* __restrict__ a, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double x = a[0], y = a[1], z = a[2];
  out[0] = (x + y + z) / 3.0;
  out[1] = sqrt(((x - y) * (x - y) + (y - z) * (y - z) + (z - x) * (z - x)) / 2.0);
}

}  // namespace
}  // namespace nof

using namespace nof;

extern "C" {

size_t nof_dipole_ws(int nbf, int norb) {
  if (nbf < 1 || norb < 1) return 0;
  return ((size_t)norb * norb * sizeof(double) + 255) / 256 * 256 +
         nof_mo_transform_ws(1, nbf, norb, NOF_F64, NOF_F64, NOF_P_F64);
}

int nof_dipole(int nbf, int norb, const double* C, const double* n, const double* d, double* mu,
               void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nbf < 1 || norb < 1) return NOF_E_DIM;
  if (norb > 1000000) return NOF_E_DIM;
  if (!C || !n || !d || !mu) return NOF_E_NULL;
  const size_t need = nof_dipole_ws(nbf, norb);
  if (!ws || ws_bytes < need) return NOF_E_WORKSPACE;
  const size_t xb = ((size_t)norb * norb * sizeof(double) + 255) / 256 * 256;
  double* X = (double*)ws;
  const int rc = nof_mo_transform(1, nbf, norb, d, NOF_F64, C, X, NOF_F64, nullptr, NOF_P_F64,
                                  (char*)ws + xb, ws_bytes - xb, stream);
  if (rc != NOF_OK) return rc;
  hipLaunchKernelGGL(k_dipole, dim3(1), dim3(256), 0, stream, norb, X, n, mu);
  return launch_status();
}

int nof_nlop_romberg(int npoint, double step, const double* mu0, const double* mu_p,
                     const double* mu_m, double* table, double* result, hipStream_t stream) {
  if (npoint < 1 || npoint > MAXPT) return NOF_E_DIM;
  if (!(step > 0.0) || !std::isfinite(step)) return NOF_E_ARG;
  if (!mu0 || !mu_p || !mu_m || !table || !result) return NOF_E_NULL;
  hipLaunchKernelGGL(k_nlop, dim3(1), dim3(64), 0, stream, npoint, step, mu0, mu_p, mu_m, table, result);
  return launch_status();
}

int nof_nlop_isotropic(const double* alpha, double* out, hipStream_t stream) {
  if (!alpha || !out) return NOF_E_NULL;
  hipLaunchKernelGGL(k_iso, dim3(1), dim3(64), 0, stream, alpha, out);
  return launch_status();
}

}  // extern "C"
