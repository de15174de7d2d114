// Occupation-number optimisation at fixed natural orbitals, FP64 (Occupation
// Number Optimization section): the ONs of each subspace Omega_g (one strong
// orbital and N_g weak ones, pairing sum rule of Eq. sum1) are generated from
// unconstrained variables by the trigonometric or the softmax mapping, the
// energy of Eq. (PNOF) is evaluated from h_pp, J and K with the coefficients of
// the chosen functional, and an L-BFGS iteration (two-loop recursion, Armijo
// backtracking) minimises it.
//
// The whole optimisation runs in one workgroup of 1024 threads (16 waves):
// every function evaluation is a matrix-vector product with M = 2J - K (one
// wave per row, lanes striding the row, butterfly reduction) plus per-orbital
// and per-subspace work; vectors live in the caller's workspace (L2 resident)
// and every reduction uses a fixed tree, so runs repeat bit for bit.  The
// loop needs no host round trip.
#include <math.h>

#include <cstdlib>

#include "common.h"

namespace nof {
namespace {

constexpr int OT = 1024;       // threads of the optimiser workgroup
constexpr int OW = OT / 64;    // waves
constexpr int LM = 8;          // L-BFGS memory

struct OccProblem {
  int norb, ns, ng, map, func;
  const int* members;          // [ns][ng+1]
  const double* hdiag; int hstride;
  const double* J; const double* K;
  const double* M;             // 2J - K (workspace)
  double* phi;                 // PNOF7: Phi_r = sqrt(n_r (1 - n_r)) (workspace)
  double* u;                   // PNOF7: u = K Phi (workspace)
  int* grp;                    // [norb] subspace of each orbital, -1 if none
  int* pos;                    // [norb] position inside the subspace (0 = strong)
};

struct OccWs {
  double *x, *g, *d, *xt, *gt, *S, *Y, *n, *nt, *dn, *v, *sy, *yy, *phi, *u;
  int *grp, *pos;
  double* M;
};

// Workspace layout (all sub-buffers 256-byte aligned).
struct OccLayout {
  size_t off[18];
  size_t total;
};
OccLayout occ_layout(int norb, int ns, int ng) {
  OccLayout L;
  const size_t nv = (size_t)ns * ng;
  const size_t sz[18] = {(size_t)norb * norb * 8, nv * 8, nv * 8, nv * 8, nv * 8, nv * 8,
                         LM * nv * 8, LM * nv * 8, (size_t)norb * 8, (size_t)norb * 8,
                         (size_t)norb * 8, (size_t)norb * 8, LM * 8, LM * 8,
                         (size_t)norb * 4, (size_t)norb * 4, (size_t)norb * 8, (size_t)norb * 8};
  size_t o = 0;
  for (int i = 0; i < 18; ++i) {
    L.off[i] = o;
    o = align256(o + sz[i]);
  }
  L.total = o;
  return L;
}
OccWs occ_ws_ptrs(void* ws, int norb, int ns, int ng) {
  const OccLayout L = occ_layout(norb, ns, ng);
  char* b = (char*)ws;
  OccWs w;
  w.M = (double*)(b + L.off[0]);
  w.x = (double*)(b + L.off[1]);
  w.g = (double*)(b + L.off[2]);
  w.d = (double*)(b + L.off[3]);
  w.xt = (double*)(b + L.off[4]);
  w.gt = (double*)(b + L.off[5]);
  w.S = (double*)(b + L.off[6]);
  w.Y = (double*)(b + L.off[7]);
  w.n = (double*)(b + L.off[8]);
  w.nt = (double*)(b + L.off[9]);
  w.dn = (double*)(b + L.off[10]);
  w.v = (double*)(b + L.off[11]);
  w.sy = (double*)(b + L.off[12]);
  w.yy = (double*)(b + L.off[13]);
  w.grp = (int*)(b + L.off[14]);
  w.pos = (int*)(b + L.off[15]);
  w.phi = (double*)(b + L.off[16]);
  w.u = (double*)(b + L.off[17]);
  return w;
}

// ---- block-wide deterministic reductions -----------------------------------
// Each wave reduces its 64 values with a butterfly (lane 0's value is kept),
// then every thread adds the OW wave results in wave order: two barriers, the
// same order on every call, the same result in every thread.
__device__ double block_sum(double a, double* red) {
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < OW; ++i) r += red[i];
  __syncthreads();
  return r;
}
__device__ double block_max(double a, double* red) {
  for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < OW; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}
__device__ double dot(const double* a, const double* b, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += OT) s = fma(a[i], b[i], s);
  return block_sum(s, red);
}

// ---- the mapping ------------------------------------------------------------
// n for subspace g from its variables x[g*ng ..]; writes n[members]
__device__ void map_group(const OccProblem& P, const double* x, double* n, int g) {
  const int* row = P.members + (long long)g * (P.ng + 1);
  const double* xg = x + (long long)g * P.ng;
  if (P.map == NOF_MAP_TRIG) {
    const double c = cos(xg[0]), s0 = sin(xg[0]);
    const double ngv = 0.5 * (1.0 + c * c);
    const double hole = 0.5 * s0 * s0;          // = 1 - n_g, without cancellation
    n[row[0]] = ngv;
    double Pp = 1.0;
    for (int i = 1; i < P.ng; ++i) {
      const double s = sin(xg[i]), ci = cos(xg[i]);
      n[row[i]] = hole * Pp * s * s;
      Pp *= ci * ci;
    }
    n[row[P.ng]] = hole * Pp;
  } else {
    // numerator and denominator scaled by exp(-m), m = max(0, max_i x_i): no
    // exponential overflows, the denominator holds a term equal to one
    double m = 0.0;
    for (int i = 0; i < P.ng; ++i) m = fmax(m, xg[i]);
    const double e0 = exp(-m);
    double den = e0;
    for (int i = 0; i < P.ng; ++i) den += exp(xg[i] - m);
    n[row[0]] = e0 / den;
    for (int i = 0; i < P.ng; ++i) n[row[1 + i]] = exp(xg[i] - m) / den;
  }
}

// dE/dx for subspace g from dE/dn (chain rule through the mapping)
__device__ void chain_group(const OccProblem& P, const double* x, const double* n,
                            const double* dn, double* gx, int g) {
  const int* row = P.members + (long long)g * (P.ng + 1);
  const double* xg = x + (long long)g * P.ng;
  double* og = gx + (long long)g * P.ng;
  const int ng = P.ng;
  if (P.map == NOF_MAP_SOFTMAX) {
    double gbar = 0.0;
    for (int i = 0; i <= ng; ++i) gbar += dn[row[i]] * n[row[i]];
    for (int i = 0; i < ng; ++i) og[i] = n[row[1 + i]] * (dn[row[1 + i]] - gbar);
    return;
  }
  const double cg = cos(xg[0]), sg = sin(xg[0]);
  const double hole = 0.5 * sg * sg;
  // n_{p_i} = hole * Pprev_i * t_i,  i = 1..ng (Pprev_1 = 1, t_ng = 1)
  double dE_dhole = 0.0;
  double Pp = 1.0;
  for (int i = 1; i <= ng; ++i) {
    const double t = i < ng ? sin(xg[i]) * sin(xg[i]) : 1.0;
    dE_dhole += dn[row[i]] * Pp * t;
    if (i < ng) Pp *= cos(xg[i]) * cos(xg[i]);
  }
  og[0] = cg * sg * (dE_dhole - dn[row[0]]);
  // reverse accumulation over theta_j, j = ng-1 .. 1
  double R = dn[row[ng]];
  for (int j = ng - 1; j >= 1; --j) {
    double Pj = 1.0;                          // prod_{l < j} cos^2 theta_l
    for (int l = 1; l < j; ++l) Pj *= cos(xg[l]) * cos(xg[l]);
    const double s = sin(xg[j]), c = cos(xg[j]);
    og[j] = 2.0 * s * c * hole * Pj * (dn[row[j]] - R);
    R = dn[row[j]] * s * s + c * c * R;
  }
}

// ---- one function evaluation: E(x), n(x), dE/dx ----------------------------
__device__ double evaluate(const OccProblem& P, const double* x, double* n, double* dn,
                           double* v, double* gx, double* red) {
  const int tid = threadIdx.x;
  for (int r = tid; r < P.norb; r += OT) n[r] = 0.0;
  __syncthreads();
  for (int g = tid; g < P.ns; g += OT) map_group(P, x, n, g);
  __syncthreads();
  const bool p7 = P.func == NOF_FUNC_PNOF7;
  if (p7) {
    for (int r = tid; r < P.norb; r += OT) P.phi[r] = sqrt(n[r] * (1.0 - n[r]));
    __syncthreads();
  }
  // v = M n (PNOF7 also u = K Phi): a wave takes RW rows at a time (their
  // loads in flight together), each row summed lane-wise over q and then
  // across the wave, the same order for any RW
  constexpr int RW = 4;
  const int lane = tid & 63, wv = tid >> 6;
  for (int r0 = wv; r0 < P.norb; r0 += RW * OW) {
    double s[RW], t[RW];
    const double* Mr[RW];
    const double* Kr[RW];
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const int r = min(r0 + j * OW, P.norb - 1);
      Mr[j] = P.M + (long long)r * P.norb;
      Kr[j] = p7 ? P.K + (long long)r * P.norb : nullptr;
      s[j] = 0.0;
      t[j] = 0.0;
    }
    for (int q = lane; q < P.norb; q += 64) {
      const double nq = n[q];
#pragma unroll
      for (int j = 0; j < RW; ++j) s[j] = fma(Mr[j][q], nq, s[j]);
      if (p7) {
        const double pq = P.phi[q];
#pragma unroll
        for (int j = 0; j < RW; ++j) t[j] = fma(Kr[j][q], pq, t[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      for (int o = 32; o > 0; o >>= 1) s[j] += __shfl_xor(s[j], o, 64);
      if (p7)
        for (int o = 32; o > 0; o >>= 1) t[j] += __shfl_xor(t[j], o, 64);
      const int r = r0 + j * OW;
      if (lane == 0 && r < P.norb) {
        v[r] = s[j];
        if (p7) P.u[r] = t[j];
      }
    }
  }
  __syncthreads();
  double e = 0.0;
  for (int r = tid; r < P.norb; r += OT) {
    const double hr = P.hdiag[(long long)r * P.hstride];
    const double nr = n[r];
    double d = 2.0 * hr + 2.0 * v[r];
    e += 2.0 * nr * hr + nr * v[r];
    const int g = P.grp[r];
    if (P.func != NOF_FUNC_HF && g >= 0) {
      const int* row = P.members + (long long)g * (P.ng + 1);
      const bool rstrong = P.pos[r] == 0;
      const double Jrr = P.J[(long long)r * P.norb + r];
      d += Jrr;
      e += nr * Jrr;
      for (int i = 0; i <= P.ng; ++i) {
        const int q = row[i];
        const double nq = n[q];
        const double Mrq = P.M[(long long)r * P.norb + q];
        d -= 2.0 * nq * Mrq;
        e -= nr * nq * Mrq;
        if (q != r) {
          const double sgn = (rstrong || i == 0) ? -1.0 : 1.0;
          const double Krq = P.K[(long long)r * P.norb + q];
          d += sgn * sqrt(nq / fmax(nr, 1e-300)) * Krq;
          e += sgn * sqrt(nr * nq) * Krq;
        }
      }
      if (p7) {
        // interpair: S_r = sum over q outside r's subspace of K_rq Phi_q;
        // E gains -Phi_r S_r per r, dE/dn_r = -2 Phi_r' S_r
        double S = P.u[r];
        for (int i = 0; i <= P.ng; ++i) S -= P.K[(long long)r * P.norb + row[i]] * P.phi[row[i]];
        const double ph = P.phi[r];
        e -= ph * S;
        d -= 2.0 * (1.0 - 2.0 * nr) / (2.0 * fmax(ph, 1e-300)) * S;
      }
    }
    dn[r] = d;
  }
  const double E = block_sum(e, red);
  for (int g = tid; g < P.ns; g += OT) chain_group(P, x, n, dn, gx, g);
  __syncthreads();
  return E;
}

__device__ bool setup(OccProblem& P, OccWs& w, int* info, double* red) {
  const int tid = threadIdx.x;
  P.grp = w.grp;
  P.pos = w.pos;
  for (int r = tid; r < P.norb; r += OT) { w.grp[r] = -1; w.pos[r] = -1; }
  __syncthreads();
  int bad = 0;
  for (int g = tid; g < P.ns; g += OT)
    for (int i = 0; i <= P.ng; ++i) {
      const int q = P.members[(long long)g * (P.ng + 1) + i];
      if (q < 0 || q >= P.norb) { bad = 1; continue; }
      w.grp[q] = g;
      w.pos[q] = i;
    }
  const double anybad = block_max((double)bad, red);
  if (anybad > 0.0) {
    if (tid == 0 && info) info[2] = NOF_E_ARG;
    return false;
  }
  return true;
}

// Several independent problems in one launch, one workgroup each (blockIdx.x
// = instance): element strides of h (diagonal base), J and K, gamma and n,
// the byte stride of the per-instance workspace, and an optional mask
// (instance skipped when active[i] == 0).  All zero: one problem.
struct OccBatch {
  long long h, jk, gamma, n, ws;
  const int* active;
};

template <class T> __device__ __forceinline__ T* shift(T* p, long long bytes) {
  return p ? (T*)((char*)p + bytes) : p;
}

// Moves P and w (and its views in P) to instance blockIdx.x; false if masked.
__device__ bool to_instance(OccProblem& P, OccWs& w, const OccBatch& ib) {
  const long long i = blockIdx.x;
  if (ib.active && !ib.active[i]) return false;
  if (i == 0) return true;
  const long long wb = i * ib.ws;
  w.x = shift(w.x, wb); w.g = shift(w.g, wb); w.d = shift(w.d, wb); w.xt = shift(w.xt, wb);
  w.gt = shift(w.gt, wb); w.S = shift(w.S, wb); w.Y = shift(w.Y, wb); w.n = shift(w.n, wb);
  w.nt = shift(w.nt, wb); w.dn = shift(w.dn, wb); w.v = shift(w.v, wb); w.sy = shift(w.sy, wb);
  w.yy = shift(w.yy, wb); w.phi = shift(w.phi, wb); w.u = shift(w.u, wb);
  w.grp = shift(w.grp, wb); w.pos = shift(w.pos, wb); w.M = shift(w.M, wb);
  P.M = w.M; P.grp = w.grp; P.pos = w.pos; P.phi = w.phi; P.u = w.u;
  P.hdiag += i * ib.h;
  P.J += i * ib.jk;
  P.K += i * ib.jk;
  return true;
}

// M = 2J - K of instance blockIdx.y (J, K stride jk; M at byte stride wsb).
__global__ void k_build_M(long long n2, const double* __restrict__ J, const double* __restrict__ K,
                          double* __restrict__ M, long long jk, long long wsb) {
  const long long y = blockIdx.y;
  J += y * jk;
  K += y * jk;
  M = shift(M, y * wsb);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x)
    M[i] = 2.0 * J[i] - K[i];
}

__global__ __launch_bounds__(OT) void k_occ_eval(OccProblem P, OccWs w, const double* gamma,
                                                 double* n_out, double* E_out, double* g_out,
                                                 int* info, OccBatch ib) {
  __shared__ double red[OT];
  if (!to_instance(P, w, ib)) return;
  {
    const long long i = blockIdx.x;
    gamma += i * ib.gamma;
    if (n_out) n_out += i * ib.n;
    if (E_out) E_out += i;
    if (g_out) g_out += i * ib.gamma;
    if (info) info += 3 * i;
  }
  if (!setup(P, w, info, red)) return;
  const double E = evaluate(P, gamma, w.n, w.dn, w.v, w.g, red);
  const int nv = P.ns * P.ng;
  for (int i = threadIdx.x; i < nv; i += OT) if (g_out) g_out[i] = w.g[i];
  for (int r = threadIdx.x; r < P.norb; r += OT) if (n_out) n_out[r] = w.n[r];
  if (threadIdx.x == 0) {
    if (E_out) *E_out = E;
    if (info) info[2] = 0;
  }
}

struct LbfgsParams {
  int maxit, maxbt;
  double tol, etol, loose, c1, step0;
  int lds;          // > 0: the iteration vectors live in that many doubles of dynamic LDS
};

// Doubles of LDS for the iteration vectors of one problem: x, g, d, xt, gt
// (nv each), the LM pairs S, Y, then n, nt, dn, v, phi, u (norb each) and
// sy, yy (LM each); 0 when they do not fit beside the reduction buffer.
constexpr size_t kOccLdsMax = 144 * 1024;
int occ_lds_doubles(int norb, int ns, int ng) {
  const size_t nv = (size_t)ns * ng;
  const size_t d = 5 * nv + 2 * (size_t)LM * nv + 6 * (size_t)norb + 2 * LM;
  return d * sizeof(double) <= kOccLdsMax ? (int)d : 0;
}

// Point the iteration vectors of w (and P's phi, u) at LDS (layout above).
__device__ void vectors_to_lds(OccProblem& P, OccWs& w, double* sm, int nv) {
  const int no = P.norb;
  double* p = sm;
  auto take = [&](long long k) { double* q = p; p += k; return q; };
  w.x = take(nv); w.g = take(nv); w.d = take(nv); w.xt = take(nv); w.gt = take(nv);
  w.S = take((long long)LM * nv); w.Y = take((long long)LM * nv);
  w.n = take(no); w.nt = take(no); w.dn = take(no); w.v = take(no); w.phi = take(no); w.u = take(no);
  w.sy = take(LM); w.yy = take(LM);
  P.phi = w.phi;
  P.u = w.u;
}

// Box of the variables: the trigonometric map is even and pi-periodic in every
// angle, so [0, pi/2]^n reaches every occupation vector once, and the points
// where E is not differentiable in the angles (a weak amplitude sqrt(n_p)
// crossing zero, a kink through PNOF5's sqrt(n_p n_q) terms) lie on its faces,
// held kTrigEdge inside.  The strong angle's lower face (n_g -> 1) is held
// kTrigStrongEdge inside: no minimum lies there (E falls linearly away from
// it, every K_gp >= 0), and closer to 0 the hole 1 - n_g is lost to rounding
// in n_g.  The softmax variables are unbounded.
constexpr double kTrigEdge = 1e-12;
constexpr double kTrigStrongEdge = 1e-6;
// bounds of variable i (row-major [ns][ng]: column 0 is the strong angle)
__device__ __forceinline__ void var_bounds(int map, int ng, int i, double& lo, double& hi) {
  if (map == NOF_MAP_TRIG) {
    lo = (i % ng) == 0 ? kTrigStrongEdge : kTrigEdge;
    hi = 0.5 * M_PI - kTrigEdge;
  } else {
    lo = -HUGE_VAL;
    hi = HUGE_VAL;
  }
}
// projection of x onto the bounds of variable i, and the projected gradient
struct VarBox {
  int map, ng;
  __device__ __forceinline__ double lo(int i) const {
    double l, h; var_bounds(map, ng, i, l, h); return l;
  }
  __device__ __forceinline__ double hi(int i) const {
    double l, h; var_bounds(map, ng, i, l, h); return h;
  }
};
// a component that pushes a variable out through a face it sits on
__device__ __forceinline__ bool held_at_face(double x, double g, double lo, double hi) {
  return (x <= lo && g > 0.0) || (x >= hi && g < 0.0);
}
__device__ __forceinline__ double proj_grad(double x, double g, double lo, double hi) {
  return held_at_face(x, g, lo, hi) ? 0.0 : g;
}

__global__ __launch_bounds__(OT) void k_occ_lbfgs(OccProblem P, OccWs w, LbfgsParams L,
                                                  double* gamma, double* n_out, double* E_out,
                                                  int* info, OccBatch ib) {
  __shared__ double red[OT];
  if (!to_instance(P, w, ib)) return;
  {
    const long long i = blockIdx.x;
    gamma += i * ib.gamma;
    if (n_out) n_out += i * ib.n;
    if (E_out) E_out += i;
    if (info) info += 3 * i;
  }
  if (!setup(P, w, info, red)) return;
  const int tid = threadIdx.x;
  const int nv = P.ns * P.ng;
  extern __shared__ double occ_sm[];
  if (L.lds > 0) vectors_to_lds(P, w, occ_sm, nv);
  const VarBox bx{P.map, P.ng};
  for (int i = tid; i < nv; i += OT) w.x[i] = fmin(fmax(gamma[i], bx.lo(i)), bx.hi(i));
  __syncthreads();
  double E = evaluate(P, w.x, w.n, w.dn, w.v, w.g, red);
  int it = 0, flat = 0, mcount = 0, head = 0;
  double gmax = 0.0;
  while (true) {
    // projected gradient: the first-order optimality measure on the box
    double gl = 0.0;
    for (int i = tid; i < nv; i += OT) gl = fmax(gl, fabs(proj_grad(w.x[i], w.g[i], bx.lo(i), bx.hi(i))));
    gmax = block_max(gl, red);
    if (it >= L.maxit || gmax <= L.tol || flat >= 2) break;
    // two-loop recursion on the projected gradient: d = H pg
    for (int i = tid; i < nv; i += OT) w.d[i] = proj_grad(w.x[i], w.g[i], bx.lo(i), bx.hi(i));
    __syncthreads();
    double alph[LM];
    for (int k = 0; k < mcount; ++k) {
      const int idx = (head - 1 - k + LM) % LM;
      const double a = dot(w.S + (long long)idx * nv, w.d, nv, red) / w.sy[idx];
      alph[k] = a;
      for (int i = tid; i < nv; i += OT) w.d[i] -= a * w.Y[(long long)idx * nv + i];
      __syncthreads();
    }
    const double scale = mcount > 0 ? w.sy[(head - 1 + LM) % LM] / w.yy[(head - 1 + LM) % LM]
                                    : L.step0 / gmax;
    for (int i = tid; i < nv; i += OT) w.d[i] *= scale;
    __syncthreads();
    for (int k = mcount - 1; k >= 0; --k) {
      const int idx = (head - 1 - k + LM) % LM;
      const double bcoef = dot(w.Y + (long long)idx * nv, w.d, nv, red) / w.sy[idx];
      for (int i = tid; i < nv; i += OT) w.d[i] += w.S[(long long)idx * nv + i] * (alph[k] - bcoef);
      __syncthreads();
    }
    // descent direction, zero on the variables held at a face
    for (int i = tid; i < nv; i += OT)
      w.d[i] = held_at_face(w.x[i], w.g[i], bx.lo(i), bx.hi(i)) ? 0.0 : -w.d[i];
    __syncthreads();
    const double gd = dot(w.g, w.d, nv, red);
    if (!(gd < 0.0)) {
      mcount = 0;
      for (int i = tid; i < nv; i += OT) w.d[i] = -proj_grad(w.x[i], w.g[i], bx.lo(i), bx.hi(i)) * (L.step0 / gmax);
      __syncthreads();
    }
    // backtracking Armijo line search, every trial point projected onto the
    // box: E_t <= E + c1 g.(x_t - x)
    double t = 1.0, Et = 0.0;
    int nb = 0;
    for (nb = 0; nb < L.maxbt; ++nb) {
      double gs = 0.0;
      for (int i = tid; i < nv; i += OT) {
        const double xt = fmin(fmax(w.x[i] + t * w.d[i], bx.lo(i)), bx.hi(i));
        w.xt[i] = xt;
        gs = fma(w.g[i], xt - w.x[i], gs);
      }
      const double gdx = block_sum(gs, red);
      Et = evaluate(P, w.xt, w.nt, w.dn, w.v, w.gt, red);
      if (Et <= E + L.c1 * gdx) break;
      t *= 0.5;
    }
    if (nb == L.maxbt) nb = L.maxbt - 1;
    // new pair s = xt - x, y = gt - g into slot head
    double* Sh = w.S + (long long)head * nv;
    double* Yh = w.Y + (long long)head * nv;
    for (int i = tid; i < nv; i += OT) {
      Sh[i] = w.xt[i] - w.x[i];
      Yh[i] = w.gt[i] - w.g[i];
    }
    __syncthreads();
    if (nb >= L.maxbt / 2) {
      mcount = 0;
    } else {
      const double sy = dot(Sh, Yh, nv, red);
      if (sy > 0.0) {
        const double yy = dot(Yh, Yh, nv, red);
        if (tid == 0) { w.sy[head] = sy; w.yy[head] = yy; }
        head = (head + 1) % LM;
        mcount = mcount < LM ? mcount + 1 : LM;
      }
    }
    double gl2 = 0.0;
    for (int i = tid; i < nv; i += OT) gl2 = fmax(gl2, fabs(proj_grad(w.xt[i], w.gt[i], bx.lo(i), bx.hi(i))));
    const double gtmax = block_max(gl2, red);
    const bool small = gtmax <= L.loose;
    flat = (small && fabs(Et - E) <= L.etol * fmax(1.0, fabs(E))) ? flat + 1 : 0;
    for (int i = tid; i < nv; i += OT) { w.x[i] = w.xt[i]; w.g[i] = w.gt[i]; }
    for (int r = tid; r < P.norb; r += OT) w.n[r] = w.nt[r];
    __syncthreads();
    E = Et;
    ++it;
  }
  for (int i = tid; i < nv; i += OT) gamma[i] = w.x[i];
  for (int r = tid; r < P.norb; r += OT) if (n_out) n_out[r] = w.n[r];
  if (tid == 0) {
    if (E_out) *E_out = E;
    if (info) {
      info[0] = it;
      info[1] = (gmax <= L.tol || flat >= 2) ? 1 : 0;
      info[2] = 0;
    }
  }
}

// cJ = 2(nn^T - Delta), cK = nn^T - Delta - Pi for the HF-like, PNOF5 or PNOF7
// functional (PNOF7: PNOF5 inside a subspace, Pi_pq = -Phi_p Phi_q between
// subspaces, Phi = sqrt(n (1 - n)))
__global__ void k_func_coeffs(int norb, int ng, int func, const double* __restrict__ n,
                              const int* __restrict__ grp, const int* __restrict__ pos,
                              double* __restrict__ cJ, double* __restrict__ cK) {
  const long long n2 = (long long)norb * norb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n2;
       i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i / norb), q = (int)(i - (long long)p * norb);
    const double nn = n[p] * n[q];
    double dl = 0.0, pi = 0.0;
    if (func != NOF_FUNC_HF && grp[p] >= 0 && grp[p] == grp[q]) {
      dl = nn;
      if (p == q) pi = n[p];
      else pi = ((pos[p] == 0 || pos[q] == 0) ? -1.0 : 1.0) * sqrt(nn);
    } else if (func == NOF_FUNC_PNOF7 && grp[p] >= 0 && grp[q] >= 0) {
      pi = -(sqrt(n[p] * (1.0 - n[p])) * sqrt(n[q] * (1.0 - n[q])));
    }
    cJ[i] = 2.0 * (nn - dl);
    cK[i] = nn - dl - pi;
  }
}

__global__ void k_group_index(int norb, int ns, int ng, const int* __restrict__ members,
                              int* __restrict__ grp, int* __restrict__ pos, int* __restrict__ bad) {
  // single block: clear, then fill
  for (int r = threadIdx.x; r < norb; r += blockDim.x) { grp[r] = -1; pos[r] = -1; }
  __syncthreads();
  for (int g = threadIdx.x; g < ns; g += blockDim.x)
    for (int i = 0; i <= ng; ++i) {
      const int q = members[(long long)g * (ng + 1) + i];
      if (q < 0 || q >= norb) {
        if (bad) bad[2] = NOF_E_ARG;
        continue;
      }
      grp[q] = g;
      pos[q] = i;
    }
}

OccProblem make_problem(int norb, int ns, int ng, const int* members, int map, int func,
                        const double* hdiag, int hstride, const double* J, const double* K,
                        const OccWs& w) {
  OccProblem P;
  P.norb = norb; P.ns = ns; P.ng = ng; P.map = map; P.func = func;
  P.members = members; P.hdiag = hdiag; P.hstride = hstride; P.J = J; P.K = K;
  P.M = w.M; P.grp = w.grp; P.pos = w.pos; P.phi = w.phi; P.u = w.u;
  return P;
}

int build_M(int norb, const double* J, const double* K, double* M, hipStream_t st, int ninst = 1,
            long long jk = 0, long long wsb = 0) {
  const long long n2 = (long long)norb * norb;
  long long g = (n2 + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_build_M, dim3((unsigned)g, ninst), dim3(256), 0, st, n2, J, K, M, jk, wsb);
  return launch_status();
}

}  // namespace

size_t occ_ws(int norb, int ns, int ng) { return occ_layout(norb, ns, ng).total; }

int occ_energy_grad(int norb, int ns, int ng, const int* members, int map, int func,
                    const double* gamma, const double* hdiag, int hstride, const double* J,
                    const double* K, double* n, double* E, double* dEdgamma, int* info, void* ws,
                    hipStream_t st) {
  OccWs w = occ_ws_ptrs(ws, norb, ns, ng);
  int rc = build_M(norb, J, K, w.M, st);
  if (rc != NOF_OK) return rc;
  OccProblem P = make_problem(norb, ns, ng, members, map, func, hdiag, hstride, J, K, w);
  hipLaunchKernelGGL(k_occ_eval, dim3(1), dim3(OT), 0, st, P, w, gamma, n, E, dEdgamma, info,
                     OccBatch{});
  return launch_status();
}


// LDS doubles for k_occ_lbfgs's vectors (0: they stay in the workspace); the
// kernel's dynamic-LDS limit is raised to that size first.  The environment
// variable NOF_OCC_VECTORS_IN_WORKSPACE=1 keeps them in the workspace at any
// size (the two placements give bit-identical results; the switch lets both
// be tested on small problems).
int lbfgs_lds(int norb, int ns, int ng) {
  const char* force_ws = std::getenv("NOF_OCC_VECTORS_IN_WORKSPACE");
  if (force_ws && force_ws[0] == '1') return 0;
  const int d = occ_lds_doubles(norb, ns, ng);
  if (d == 0) return 0;
  const size_t bytes = (size_t)d * sizeof(double);
  if (bytes > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_occ_lbfgs),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return d;
}

int occ_optimize(int norb, int ns, int ng, const int* members, int map, int func,
                 const double* hdiag, int hstride, const double* J, const double* K,
                 double* gamma, double* n, double* E, int* info, int maxit, double tol, void* ws,
                 hipStream_t st) {
  OccWs w = occ_ws_ptrs(ws, norb, ns, ng);
  int rc = build_M(norb, J, K, w.M, st);
  if (rc != NOF_OK) return rc;
  OccProblem P = make_problem(norb, ns, ng, members, map, func, hdiag, hstride, J, K, w);
  LbfgsParams L;
  L.maxit = maxit; L.maxbt = 50; L.tol = tol; L.etol = 1e-14; L.loose = 1e-5; L.c1 = 1e-4;
  L.step0 = 0.1;
  L.lds = lbfgs_lds(norb, ns, ng);
  hipLaunchKernelGGL(k_occ_lbfgs, dim3(1), dim3(OT), (size_t)L.lds * sizeof(double), st, P, w, L, gamma,
                     n, E, info, OccBatch{});
  return launch_status();
}

size_t occ_ws_stride(int norb, int ns, int ng) { return align256(occ_layout(norb, ns, ng).total); }

int occ_batched(int ninst, const int* active, int norb, int ns, int ng, const int* members, int map,
                int func, const double* hdiag, int hstride, long long hinst, const double* J,
                const double* K, long long jkinst, double* gamma, double* n, double* E, int* info,
                int maxit, double tol, void* ws, hipStream_t st) {
  const size_t wsb = occ_ws_stride(norb, ns, ng);
  OccWs w = occ_ws_ptrs(ws, norb, ns, ng);
  int rc = build_M(norb, J, K, w.M, st, ninst, jkinst, (long long)wsb);
  if (rc != NOF_OK) return rc;
  OccProblem P = make_problem(norb, ns, ng, members, map, func, hdiag, hstride, J, K, w);
  const OccBatch ib{hinst, jkinst, (long long)ns * ng, norb, (long long)wsb, active};
  if (maxit > 0) {
    LbfgsParams L;
    L.maxit = maxit; L.maxbt = 50; L.tol = tol; L.etol = 1e-14; L.loose = 1e-5; L.c1 = 1e-4;
    L.step0 = 0.1;
    L.lds = lbfgs_lds(norb, ns, ng);
    hipLaunchKernelGGL(k_occ_lbfgs, dim3(ninst), dim3(OT), (size_t)L.lds * sizeof(double), st, P, w, L,
                       gamma, n, E, info, ib);
  } else {
    hipLaunchKernelGGL(k_occ_eval, dim3(ninst), dim3(OT), 0, st, P, w, gamma, n, E,
                       (double*)nullptr, info, ib);
  }
  return launch_status();
}

int functional_coeffs(int norb, int ns, int ng, const int* members, int func, const double* n,
                      double* cJ, double* cK, void* ws, int* bad, hipStream_t st) {
  OccWs w = occ_ws_ptrs(ws, norb, ns, ng);
  hipLaunchKernelGGL(k_group_index, dim3(1), dim3(1024), 0, st, norb, ns, ng, members, w.grp,
                     w.pos, bad);
  int rc = launch_status();
  if (rc != NOF_OK) return rc;
  const long long n2 = (long long)norb * norb;
  long long g = (n2 + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_func_coeffs, dim3((unsigned)g), dim3(256), 0, st, norb, ng, func, n, w.grp,
                     w.pos, cJ, cK);
  return launch_status();
}

}  // namespace nof
