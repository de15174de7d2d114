// Iterative diagonalization of the generalized pseudo-Fockian (Natural
// Orbital Optimization: the orbital-optimisation scheme selected by
// IORBOPT = 1).
//
// At the minimum lambda is symmetric; a symmetric F whose off-diagonal
// elements are the asymmetry of lambda is then diagonal, and away from the
// minimum its eigenvectors give the next orbitals.  F_pq = F_qp =
// s_pq (lambda_qp - lambda_pq), s_pq = +1 when diag_p <= diag_q (p < q),
// clamped to [-maxoff, maxoff]; F_pp = diag_p (lambda_pp when no diagonal is
// given).
//
// Eigensolver: cyclic two-sided Jacobi with the round-robin ordering of
// Brent and Luk (n/2 disjoint rotations per step, n-1 steps per sweep).  One
// launch per step: a thread owns a 2x2 block of A (pair i of rows, pair j of
// columns, i <= j, and the mirrored block) and reads it from the previous
// buffer, so no two threads touch the same element; another thread set owns
// (row, pair) of the accumulated rotations V.  Each rotation has
// |angle| <= pi/4 (Golub and Van Loan, symmetric Schur decomposition), which
// keeps every eigenvector near the orbital it starts from.  An odd order is
// padded with a decoupled zero row and column.  Sweeps stop when
// max|A_pq| (p != q) <= 1e-14 max|A_pp| (checked on the host between sweeps).
//
// Afterwards the eigenvectors are matched to the orbitals greedily by
// overlap (k_assign): V column r(k) = +-eigenvector k with V_rr >= 0, eig_r =
// its eigenvalue.
#include <algorithm>
#include <cmath>
#include <new>

#include "common.h"

namespace nof {
namespace {

constexpr int DG_THR = 256;
constexpr int DG_MAX_SWEEPS = 40;
constexpr double DG_TOL = 1e-14;

inline int dg_grid(long long n) {
  long long g = (n + DG_THR - 1) / DG_THR;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

__global__ void k_pseudo_fock(int norb, int np, const double* __restrict__ lam,
                              const double* __restrict__ diag, double maxoff, double* __restrict__ F) {
  const long long nn = (long long)np * np;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i / np), q = (int)(i - (long long)p * np);
    double v = 0.0;
    if (p < norb && q < norb) {
      const int a = min(p, q), b = max(p, q);
      const double da = diag ? diag[a] : lam[(long long)a * norb + a];
      if (a == b) {
        v = da;
      } else {
        const double db = diag ? diag[b] : lam[(long long)b * norb + b];
        const double s = da <= db ? 1.0 : -1.0;
        v = s * (lam[(long long)b * norb + a] - lam[(long long)a * norb + b]);
        v = fmin(fmax(v, -maxoff), maxoff);
      }
    }
    F[i] = v;
  }
}

__global__ void k_identity(int np, double* __restrict__ V) {
  const long long nn = (long long)np * np;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i / np), q = (int)(i - (long long)p * np);
    V[i] = p == q ? 1.0 : 0.0;
  }
}

// position of player j in round k of the circle method (player 0 fixed)
__device__ __forceinline__ int rr_pos(int j, int k, int np) {
  return j == 0 ? 0 : ((j - 1 + k) % (np - 1)) + 1;
}
__device__ __forceinline__ void rr_pair(int i, int k, int np, int& p, int& q) {
  const int a = rr_pos(i, k, np), b = rr_pos(np - 1 - i, k, np);
  p = min(a, b);
  q = max(a, b);
}
// (c, s) of the rotation J = [[c, s], [-s, c]] on (p, q) with (J^T A J)_pq = 0
__device__ __forceinline__ void jrot(double app, double aqq, double apq, double& c, double& s) {
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (aqq - app) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// One round k: A_out = J^T A_in J for the np/2 rotations of the round, V <- V J.
__global__ __launch_bounds__(DG_THR) void k_jacobi_step(int np, int k, const double* __restrict__ Ain,
                                                        double* __restrict__ Aout, double* __restrict__ V) {
  const int nh = np / 2;
  const long long nA = (long long)nh * nh;
  const long long total = nA + (long long)np * nh;
  for (long long u = blockIdx.x * (long long)blockDim.x + threadIdx.x; u < total;
       u += (long long)gridDim.x * blockDim.x) {
    if (u < nA) {
      const int i = (int)(u / nh), j = (int)(u - (long long)i * nh);
      if (i > j) continue;
      int pi, qi, pj, qj;
      rr_pair(i, k, np, pi, qi);
      rr_pair(j, k, np, pj, qj);
      double ci, si, cj, sj;
      jrot(Ain[(long long)pi * np + pi], Ain[(long long)qi * np + qi], Ain[(long long)pi * np + qi], ci, si);
      jrot(Ain[(long long)pj * np + pj], Ain[(long long)qj * np + qj], Ain[(long long)pj * np + qj], cj, sj);
      const double m00 = Ain[(long long)pi * np + pj], m01 = Ain[(long long)pi * np + qj];
      const double m10 = Ain[(long long)qi * np + pj], m11 = Ain[(long long)qi * np + qj];
      const double l00 = ci * m00 - si * m10, l01 = ci * m01 - si * m11;
      const double l10 = si * m00 + ci * m10, l11 = si * m01 + ci * m11;
      double n00 = l00 * cj - l01 * sj, n01 = l00 * sj + l01 * cj;
      double n10 = l10 * cj - l11 * sj, n11 = l10 * sj + l11 * cj;
      if (i == j) {
        n01 = 0.0;
        n10 = 0.0;
      }
      Aout[(long long)pi * np + pj] = n00;
      Aout[(long long)pi * np + qj] = n01;
      Aout[(long long)qi * np + pj] = n10;
      Aout[(long long)qi * np + qj] = n11;
      if (i != j) {
        Aout[(long long)pj * np + pi] = n00;
        Aout[(long long)qj * np + pi] = n01;
        Aout[(long long)pj * np + qi] = n10;
        Aout[(long long)qj * np + qi] = n11;
      }
    } else {
      const long long v = u - nA;
      const int r = (int)(v / nh), i = (int)(v - (long long)r * nh);
      int p, q;
      rr_pair(i, k, np, p, q);
      double c, s;
      jrot(Ain[(long long)p * np + p], Ain[(long long)q * np + q], Ain[(long long)p * np + q], c, s);
      double* row = V + (long long)r * np;
      const double vp = row[p], vq = row[q];
      row[p] = vp * c - vq * s;
      row[q] = vp * s + vq * c;
    }
  }
}

// out[0] = max_{p != q} |A_pq|, out[1] = max_p |A_pp| over the first norb rows
// and columns; one workgroup, fixed order.
__global__ __launch_bounds__(1024) void k_offdiag(int norb, int np, const double* __restrict__ A,
                                                  double* __restrict__ out) {
  __shared__ double ro[1024], rd[1024];
  double mo = 0.0, md = 0.0;
  const long long nn = (long long)norb * norb;
  for (long long i = threadIdx.x; i < nn; i += 1024) {
    const int p = (int)(i / norb), q = (int)(i - (long long)p * norb);
    const double a = fabs(A[(long long)p * np + q]);
    if (p == q) md = fmax(md, a);
    else mo = fmax(mo, a);
  }
  ro[threadIdx.x] = mo;
  rd[threadIdx.x] = md;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ro[threadIdx.x] = fmax(ro[threadIdx.x], ro[threadIdx.x + w]);
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ro[0];
    out[1] = rd[0];
  }
}

// Greedy overlap matching of eigenvectors (columns k of W) to orbitals (rows
// r): pairs in decreasing |W_rk| (ties: smaller r, then smaller k), each
// taken while both are free.  Computed as rounds of mutual best choices
// (every free column's best free row, every free row's best free column; a
// pair that chose each other is the largest of all pairs touching either, so
// the greedy rule takes it too); each round takes at least the largest free
// pair, so at most norb rounds.  perm[k] = orbital of eigenvector k;
// info[0] = sweeps, info[1] = rounds.  One workgroup.
__global__ __launch_bounds__(1024) void k_assign(int norb, int np, const double* __restrict__ W,
                                                 int* __restrict__ perm, int* __restrict__ used,
                                                 int* __restrict__ best_row, int* __restrict__ best_col,
                                                 int* __restrict__ info, int sweeps) {
  __shared__ int more;
  const int tid = threadIdx.x;
  for (int i = tid; i < norb; i += 1024) {
    perm[i] = -1;
    used[i] = 0;
  }
  __syncthreads();
  int rounds = 0;
  for (;;) {
    ++rounds;
    for (int k = tid; k < norb; k += 1024) {
      if (perm[k] >= 0) continue;
      int br = -1;
      double bv = -1.0;
      for (int r = 0; r < norb; ++r) {
        if (used[r]) continue;
        const double a = fabs(W[(long long)r * np + k]);
        if (a > bv) {
          bv = a;
          br = r;
        }
      }
      best_row[k] = br;
    }
    for (int r = tid; r < norb; r += 1024) {
      if (used[r]) continue;
      int bc = -1;
      double bv = -1.0;
      const double* row = W + (long long)r * np;
      for (int k = 0; k < norb; ++k) {
        if (perm[k] >= 0) continue;
        const double a = fabs(row[k]);
        if (a > bv) {
          bv = a;
          bc = k;
        }
      }
      best_col[r] = bc;
    }
    __syncthreads();
    for (int k = tid; k < norb; k += 1024) {
      if (perm[k] >= 0) continue;
      const int r = best_row[k];
      if (best_col[r] == k) {
        perm[k] = r;
        used[r] = 1;
      }
    }
    if (tid == 0) more = 0;
    __syncthreads();
    for (int k = tid; k < norb; k += 1024)
      if (perm[k] < 0) more = 1;          // every writer stores the same value
    __syncthreads();
    if (!more || rounds >= norb) break;
  }
  if (tid == 0 && info) {
    info[0] = sweeps;
    info[1] = rounds;
  }
}

// V[r][perm k] = sign_k W[r][k], eig[perm k] = A[k][k], sign_k making
// V[perm k][perm k] >= 0.
__global__ void k_permute(int norb, int np, const double* __restrict__ W, const double* __restrict__ A,
                          const int* __restrict__ perm, double* __restrict__ V, double* __restrict__ eig) {
  const long long nn = (long long)norb * norb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / norb), k = (int)(i - (long long)r * norb);
    const int c = perm[k];
    const double sg = W[(long long)c * np + k] < 0.0 ? -1.0 : 1.0;
    V[(long long)r * norb + c] = sg * W[(long long)r * np + k];
    if (r == 0 && eig) eig[c] = A[(long long)k * np + k];
  }
}

struct DiagLayout {
  int np;
  size_t a0, a1, w, perm, used, brow, bcol, scal, total;
};
DiagLayout diag_layout(int norb) {
  DiagLayout L;
  L.np = norb + (norb & 1);
  const size_t m = (size_t)L.np * L.np * sizeof(double);
  size_t o = 0;
  L.a0 = o;   o += align256(m);
  L.a1 = o;   o += align256(m);
  L.w = o;    o += align256(m);
  L.perm = o; o += align256((size_t)norb * sizeof(int));
  L.used = o; o += align256((size_t)norb * sizeof(int));
  L.brow = o; o += align256((size_t)norb * sizeof(int));
  L.bcol = o; o += align256((size_t)norb * sizeof(int));
  L.scal = o; o += 256;
  L.total = o;
  return L;
}

}  // namespace
}  // namespace nof

using namespace nof;

extern "C" {

size_t nof_pseudo_fock_diag_ws(int norb) {
  if (norb < 1 || norb > (1 << 16)) return 0;
  return diag_layout(norb).total;
}

int nof_pseudo_fock_diag(int norb, const double* lambda, const double* diag, double maxoff, double* V,
                         double* eig, int* info, void* ws, size_t ws_bytes, hipStream_t stream) {
  try {
    if (norb < 1 || norb > (1 << 16)) return NOF_E_DIM;
    if (!lambda || !V) return NOF_E_NULL;
    if (!(maxoff > 0.0)) return NOF_E_ARG;
    const DiagLayout L = diag_layout(norb);
    if (!ws || ws_bytes < L.total) return NOF_E_WORKSPACE;
    char* w = (char*)ws;
    double* A = (double*)(w + L.a0);
    double* B = (double*)(w + L.a1);
    double* W = (double*)(w + L.w);
    int* perm = (int*)(w + L.perm);
    int* used = (int*)(w + L.used);
    int* brow = (int*)(w + L.brow);
    int* bcol = (int*)(w + L.bcol);
    double* scal = (double*)(w + L.scal);
    const int np = L.np;
    const long long nn = (long long)np * np;
    hipLaunchKernelGGL(k_pseudo_fock, dim3(dg_grid(nn)), dim3(DG_THR), 0, stream, norb, np, lambda, diag,
                       maxoff, A);
    int rc = launch_status();
    if (rc != NOF_OK) return rc;
    hipLaunchKernelGGL(k_identity, dim3(dg_grid(nn)), dim3(DG_THR), 0, stream, np, W);
    if ((rc = launch_status()) != NOF_OK) return rc;
    const long long nh = np / 2;
    const int step_grid = dg_grid(nh * nh + (long long)np * nh);
    int sweeps = 0;
    bool converged = false;
    for (;;) {
      hipLaunchKernelGGL(k_offdiag, dim3(1), dim3(1024), 0, stream, norb, np, A, scal);
      if ((rc = launch_status()) != NOF_OK) return rc;
      double h[2];
      if (hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess)
        return NOF_E_HIP;
      if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return NOF_E_ARG;
      if (h[0] <= DG_TOL * h[1] || h[0] == 0.0) {
        converged = true;
        break;
      }
      if (sweeps == DG_MAX_SWEEPS) break;
      for (int k = 0; k < np - 1; ++k) {
        hipLaunchKernelGGL(k_jacobi_step, dim3(step_grid), dim3(DG_THR), 0, stream, np, k, A, B, W);
        if ((rc = launch_status()) != NOF_OK) return rc;
        std::swap(A, B);
      }
      ++sweeps;
    }
    hipLaunchKernelGGL(k_assign, dim3(1), dim3(1024), 0, stream, norb, np, W, perm, used, brow, bcol, info,
                       converged ? sweeps : -1);
    if ((rc = launch_status()) != NOF_OK) return rc;
    hipLaunchKernelGGL(k_permute, dim3(dg_grid((long long)norb * norb)), dim3(DG_THR), 0, stream, norb, np,
                       W, A, perm, V, eig);
    if ((rc = launch_status()) != NOF_OK) return rc;
    return converged ? NOF_OK : NOF_E_NOT_CONVERGED;
  } catch (const std::bad_alloc&) {
    return NOF_E_INTERNAL;
  } catch (...) {
    return NOF_E_INTERNAL;
  }
}

}  // extern "C"
