// The alternating NO + ON optimisation to convergence (Theory: the energy is
// minimised separately over occupations and orbitals; Occupation Number
// Optimization; Natural Orbital Optimization), driven from the host through
// the library's own entry points on one stream.
//
// Outer iteration: ON step at fixed orbitals (transform, h, J, K, L-BFGS on
// gamma, coefficients), then a NO sweep of up to no_steps ADAM steps on the
// orbital gradient g = 4(lambda - lambda^T) with U = exp(y), C <- C U (or,
// with orbopt = 1, steps of the iterative diagonalization of the generalized
// pseudo-Fockian: U = its eigenvectors).  A sweep
// stops once max|lambda - lambda^T| <= tol_lambda; the run stops when a sweep
// ended that way and E moved by at most tol_energy since the previous outer
// iteration.  ADAM moments persist over the whole run (one step counter).
// Per NO step the host reads two scalars (E and the asymmetry of lambda).
#include <algorithm>
#include <cmath>
#include <new>

#include "common.h"

namespace nof {
namespace {

// max_pq |L_pq - L_qp| of an n x n FP64 matrix, one workgroup.
__global__ void k_asym(int n, const double* __restrict__ L, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  const long long nn = (long long)n * n;
  for (long long i = threadIdx.x; i < nn; i += blockDim.x) {
    const long long p = i / n, q = i - p * n;
    if (q > p) m = fmax(m, fabs(L[p * n + q] - L[q * n + p]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

struct SolveLayout {
  size_t b, D, h, J, K, lam, g, cJ, cK, m, v, y, U, Cn, n, dg, scal, info, scratch, total;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Storage of b for a precision mode.
int b_type(int prec) { return prec == NOF_P_F64 ? NOF_F64 : NOF_F32; }

SolveLayout solve_layout(int naux, int nbf, int norb, int ns, int ng, int Bt, int prec) {
  SolveLayout L{};
  const size_t n2 = (size_t)norb * norb * sizeof(double);
  const int bt = b_type(prec);
  size_t o = 0;
  L.b = o;   o += a256((size_t)naux * norb * norb * (bt == NOF_F64 ? 8 : 4));
  L.D = o;   o += a256((size_t)naux * norb * sizeof(double));
  L.h = o;   o += a256(n2);
  L.J = o;   o += a256(n2);
  L.K = o;   o += a256(n2);
  L.lam = o; o += a256(n2);
  L.g = o;   o += a256(n2);
  L.cJ = o;  o += a256(n2);
  L.cK = o;  o += a256(n2);
  L.m = o;   o += a256(n2);
  L.v = o;   o += a256(n2);
  L.y = o;   o += a256(n2);
  L.U = o;   o += a256(n2);
  L.Cn = o;  o += a256((size_t)nbf * norb * sizeof(double));
  L.n = o;   o += a256((size_t)norb * sizeof(double));
  L.dg = o;  o += a256((size_t)norb * sizeof(double));   // pseudo-Fockian diagonal (orbopt 1)
  L.scal = o; o += 256;                      // E, E_on, asym, orthonormality error
  L.info = o; o += 256;                      // ON info
  L.scratch = o;
  size_t s = 0;
  s = std::max(s, nof_mo_transform_ws(naux, nbf, norb, Bt, bt, prec));
  s = std::max(s, nof_mo_transform_ws(1, nbf, norb, NOF_F64, NOF_F64, NOF_P_F64));
  s = std::max(s, nof_jk_diag_ws(naux, norb, bt));
  s = std::max(s, nof_gen_fock_ws(naux, norb, bt, prec));
  s = std::max(s, nof_expm_antisym_ws(norb));
  s = std::max(s, nof_rotate_orbitals_ws(nbf, norb));
  s = std::max(s, nof_occ_ws(norb, ns, ng));
  s = std::max(s, nof_orthonormalize_ws(nbf, norb));
  s = std::max(s, nof_energy_ws(norb));
  s = std::max(s, nof_pseudo_fock_diag_ws(norb));
  L.total = L.scratch + a256(s);
  return L;
}

}  // namespace
}  // namespace nof

using namespace nof;

extern "C" {

size_t nof_solve_ws(int naux, int nbf, int norb, int ns, int ng, int Bt, int prec) {
  if (naux < 1 || nbf < 1 || norb < 1 || ns < 1 || ng < 1) return 0;
  if (prec != NOF_P_F64 && prec != NOF_P_F32 && prec != NOF_P_BF16X10) return 0;
  if (nof_mo_transform_ws(naux, nbf, norb, Bt, b_type(prec), prec) == 0) return 0;
  return solve_layout(naux, nbf, norb, ns, ng, Bt, prec).total;
}

int nof_solve(int naux, int nbf, int norb, const void* B, int Bt, const double* H, double* C,
              int ns, int ng, const int* members, int map, int func, double* gamma, double* n_out,
              int prec, const nof_solve_params* p, nof_solve_result* res, void* ws,
              size_t ws_bytes, hipStream_t stream) {
  try {
    if (!B || !H || !C || !members || !gamma || !p || !res) return NOF_E_NULL;
    if (p->max_outer < 1 || p->no_steps < 1 || p->on_maxit < 0 || !(p->lr > 0.0) ||
        !(p->tol_orth >= 0.0) || (p->orbopt == 1 && !(p->maxoff > 0.0)))
      return NOF_E_ARG;
    if (p->orbopt == 1 && nof_pseudo_fock_diag_ws(norb) == 0) return NOF_E_DIM;
    const size_t need = nof_solve_ws(naux, nbf, norb, ns, ng, Bt, prec);
    if (need == 0) return NOF_E_DIM;
    if (!ws || ws_bytes < need) return NOF_E_WORKSPACE;
    const SolveLayout L = solve_layout(naux, nbf, norb, ns, ng, Bt, prec);
    char* w = (char*)ws;
    const int bt = b_type(prec);
    void* b = w + L.b;
    double* D = (double*)(w + L.D);
    double *h = (double*)(w + L.h), *J = (double*)(w + L.J), *K = (double*)(w + L.K);
    double *lam = (double*)(w + L.lam), *g = (double*)(w + L.g);
    double *cJ = (double*)(w + L.cJ), *cK = (double*)(w + L.cK);
    double *m = (double*)(w + L.m), *v = (double*)(w + L.v), *y = (double*)(w + L.y);
    double *U = (double*)(w + L.U), *Cn = (double*)(w + L.Cn);
    double* n = (double*)(w + L.n);
    double* dg = (double*)(w + L.dg);
    bool have_dg = false;
    double* scal = (double*)(w + L.scal);            // [0] E, [1] E of the ON step, [2] asym
    int* info = (int*)(w + L.info);
    void* scr = w + L.scratch;
    const size_t sbytes = L.total - L.scratch;
    const size_t n2 = (size_t)norb * norb * sizeof(double);

    *res = nof_solve_result{};
    res->status = NOF_OK;
#define NOF_STEP(expr)                     \
  do {                                     \
    const int rc_ = (expr);                \
    if (rc_ != NOF_OK) {                   \
      res->status = rc_;                   \
      return rc_;                          \
    }                                      \
  } while (0)

    NOF_STEP(hipMemsetAsync(m, 0, n2, stream) == hipSuccess ? NOF_OK : NOF_E_HIP);
    NOF_STEP(hipMemsetAsync(v, 0, n2, stream) == hipSuccess ? NOF_OK : NOF_E_HIP);
    auto integrals = [&](bool want_J) -> int {
      int rc = nof_mo_transform(naux, nbf, norb, B, Bt, C, b, bt, D, prec, scr, sbytes, stream);
      if (rc != NOF_OK) return rc;
      rc = nof_mo_transform(1, nbf, norb, H, NOF_F64, C, h, NOF_F64, nullptr, NOF_P_F64, scr, sbytes,
                            stream);
      if (rc != NOF_OK || !want_J) return rc;
      return nof_jk_diag(naux, norb, b, bt, D, J, K, scr, sbytes, stream);
    };
    double host[3];
    int hinfo[3];
    double E_prev = 0.0;
    bool have_prev = false;
    int t_global = 0;
    for (int outer = 0; outer < p->max_outer; ++outer) {
      // ON step at fixed orbitals
      NOF_STEP(integrals(true));
      if (p->on_maxit > 0) {
        NOF_STEP(nof_occ_optimize(norb, ns, ng, members, map, func, h, norb + 1, J, K, gamma, n,
                                  scal + 1, info, p->on_maxit, p->on_tol, scr, sbytes, stream));
        NOF_STEP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, stream) == hipSuccess
                     ? NOF_OK : NOF_E_HIP);
      } else {
        NOF_STEP(nof_occ_energy_grad(norb, ns, ng, members, map, func, gamma, h, norb + 1, J, K, n,
                                     scal + 1, nullptr, info, scr, sbytes, stream));
        NOF_STEP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, stream) == hipSuccess
                     ? NOF_OK : NOF_E_HIP);
      }
      NOF_STEP(hipStreamSynchronize(stream) == hipSuccess ? NOF_OK : NOF_E_HIP);
      if (hinfo[2] != NOF_OK) NOF_STEP(hinfo[2]);
      bool on_ok = true;
      if (p->on_maxit > 0) {
        res->on_iters += hinfo[0];
        on_ok = hinfo[1] != 0;
        if (!on_ok) ++res->on_unconverged;
      }
      NOF_STEP(nof_functional_coeffs(norb, ns, ng, members, func, n, cJ, cK, nullptr, scr, sbytes,
                                     stream));
      // NO sweep at fixed occupations
      for (int t = 0; t < p->no_steps; ++t) {
        if (t > 0) NOF_STEP(integrals(false));
        NOF_STEP(nof_jk_diag(naux, norb, b, bt, D, J, nullptr, scr, sbytes, stream));
        NOF_STEP(nof_gen_fock(naux, norb, b, bt, D, n, h, cJ, cK, lam, g, K, prec, scr, sbytes,
                              stream));
        NOF_STEP(nof_energy(norb, n, h, J, K, cJ, cK, scal, scr, sbytes, stream));
        hipLaunchKernelGGL(k_asym, dim3(1), dim3(256), 0, stream, norb, lam, scal + 2);
        NOF_STEP(launch_status());
        NOF_STEP(hipMemcpyAsync(host, scal, sizeof(host), hipMemcpyDeviceToHost, stream) == hipSuccess
                     ? NOF_OK : NOF_E_HIP);
        NOF_STEP(hipStreamSynchronize(stream) == hipSuccess ? NOF_OK : NOF_E_HIP);
        res->E = host[0];
        res->asym = host[2];
        if (!std::isfinite(host[0]) || !std::isfinite(host[2])) NOF_STEP(NOF_E_NOT_CONVERGED);
        if (host[2] <= p->tol_lambda) break;
        ++t_global;
        ++res->no_steps;
        if (p->orbopt == 1) {
          // iterative diagonalization: U = eigenvectors of the pseudo-Fockian,
          // whose eigenvalues are the next step's diagonal
          NOF_STEP(nof_pseudo_fock_diag(norb, lam, have_dg ? dg : nullptr, p->maxoff, U, dg, nullptr, scr,
                                        sbytes, stream));
          have_dg = true;
        } else {
          NOF_STEP(nof_adam_step(norb, g, m, v, t_global, p->lr, p->beta1, p->beta2, p->eps, y, stream));
          NOF_STEP(nof_expm_antisym(norb, y, U, scr, sbytes, stream));
        }
        NOF_STEP(nof_rotate_orbitals(nbf, norb, C, U, Cn, scr, sbytes, stream));
        NOF_STEP(hipMemcpyAsync(C, Cn, (size_t)nbf * norb * sizeof(double), hipMemcpyDeviceToDevice,
                                stream) == hipSuccess ? NOF_OK : NOF_E_HIP);
      }
      // orthonormality of the orbitals after the sweep, repaired past tol_orth
      NOF_STEP(nof_orthonormalize(nbf, norb, C, nullptr, p->tol_orth, scal + 3, scr, sbytes, stream));
      double orth = 0.0;
      NOF_STEP(hipMemcpyAsync(&orth, scal + 3, sizeof(double), hipMemcpyDeviceToHost, stream) == hipSuccess
                   ? NOF_OK : NOF_E_HIP);
      NOF_STEP(hipStreamSynchronize(stream) == hipSuccess ? NOF_OK : NOF_E_HIP);
      res->orth = std::max(res->orth, orth);
      res->outer = outer + 1;
      if (on_ok && res->asym <= p->tol_lambda && have_prev && std::fabs(res->E - E_prev) <= p->tol_energy) {
        res->converged = 1;
        break;
      }
      E_prev = res->E;
      have_prev = true;
    }
    if (n_out)
      NOF_STEP(hipMemcpyAsync(n_out, n, (size_t)norb * sizeof(double), hipMemcpyDeviceToDevice, stream) ==
                       hipSuccess ? NOF_OK : NOF_E_HIP);
#undef NOF_STEP
    return NOF_OK;
  } catch (const std::bad_alloc&) {
    return NOF_E_INTERNAL;
  } catch (...) {
    return NOF_E_INTERNAL;
  }
}

}  // extern "C"
