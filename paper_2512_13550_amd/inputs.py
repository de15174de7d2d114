"""Seeded synthetic inputs for the density-fitted JK / generalized-Fock path.

This module is shared by the CPU oracle's tests and by the HIP path's tests and
benchmark.  It draws random numbers and lays them out; it contains none of the
method's arithmetic (no transform, no J/K, no Fock, no energy).

Stand-ins: the paper's workloads are molecules (integrals from libcint) and a
1000-atom hydrogen chain.  None of those integrals are available, so every
tensor here is synthetic with the shapes and structure of those inputs:

* ``B[P][mu][nu]``: the three-index density-fitting tensor of the RI route
  (Computational Details / Single Point Energy: ERITYP='RI').  Symmetric in
  (mu, nu); upper triangle drawn N(0, 1/Naux), mirrored, then damped by
  exp(-|mu-nu|/L) so that it decays away from the diagonal like integrals over
  a chain of atoms.  Each P slab has its own seeded stream, so slabs can be
  drawn independently (streamed) in any order.
* ``C``: orthonormal NO coefficients (columns are orbitals), Q of a Gaussian
  QR with the sign of diag(R) folded in.
* ``H``: symmetric one-electron matrix in the AO basis, N(0,1) off-diagonal,
  diagonal U(-2, 0).
* occupations: strong orbitals 1-U(1e-3,5e-2), weak U(0,2e-2), rescaled to
  sum to the number of strong orbitals (electron pairs).
"""
from __future__ import annotations

import dataclasses
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np


# --------------------------------------------------------------------------
# Workload shapes
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nbf: int
    naux: int
    norb: int
    decay: float          # L in exp(-|mu-nu|/L)
    nstrong: int          # number of strongly occupied orbitals (electron pairs)
    ng: int               # weak orbitals per strong orbital (N_g)
    seed: int
    iters: int = 1


WORKLOADS = {
    # tiny parity instance: Nbf=48, Naux=192, Norb=48, 12 strong orbitals
    "tiny": Workload("tiny", 48, 192, 48, 8.0, 12, 3, 0),
    # FP64 vs FP32 build, 10 orbital-optimisation iterations
    "c500": Workload("c500", 500, 2000, 500, 25.0, 125, 3, 1001, iters=10),
    # 1000-hydrogen-chain-shaped precision instance (1000 electrons)
    "chain1000": Workload("chain1000", 1000, 4000, 1000, 25.0, 500, 1, 2001),
    # finite-field batch: 25 instances sharing one B
    "field300": Workload("field300", 300, 1200, 300, 25.0, 75, 3, 3001),
}


# --------------------------------------------------------------------------
# B tensor
# --------------------------------------------------------------------------
def _slab_rng(seed: int, P: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(P), 0xB])))


_DAMP_CACHE: dict = {}


def _damping(nbf: int, decay: float) -> np.ndarray:
    key = (nbf, float(decay))
    d = _DAMP_CACHE.get(key)
    if d is None:
        idx = np.arange(nbf)
        d = np.exp(-np.abs(idx[:, None] - idx[None, :]) / decay)
        _DAMP_CACHE[key] = d
    return d


def make_B_slab(seed: int, P: int, nbf: int, naux: int, decay: float,
                dtype=np.float64) -> np.ndarray:
    """One slab B[P] (nbf x nbf, symmetric), reproducible from (seed, P) alone.

    An nbf x nbf standard-normal draw; its upper triangle (with the diagonal)
    is kept and mirrored, scaled to variance 1/naux, then damped."""
    rng = _slab_rng(seed, P)
    G = rng.standard_normal((nbf, nbf))
    U = np.triu(G)
    S = U + U.T
    S[np.diag_indices(nbf)] *= 0.5
    S *= _damping(nbf, decay) * (1.0 / math.sqrt(naux))
    return S.astype(dtype, copy=False)


def make_B(seed: int, nbf: int, naux: int, decay: float, dtype=np.float64,
           P_range=None, threads: int = 8) -> np.ndarray:
    """B[P][mu][nu] for P in P_range (default all), drawn slab by slab."""
    lo, hi = (0, naux) if P_range is None else P_range
    out = np.empty((hi - lo, nbf, nbf), dtype=dtype)

    def fill(P):
        out[P - lo] = make_B_slab(seed, P, nbf, naux, decay, dtype)

    if threads > 1 and hi - lo > 8:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, range(lo, hi)))
    else:
        for P in range(lo, hi):
            fill(P)
    return out


def make_B_grid(nbf: int, naux: int, seed: int = 0, sigma: float = 1.5,
                width: float = 0.8) -> np.ndarray:
    """Kernel-on-grid three-index tensor with physical positivity.

    B^P_{mu nu} = sum_g L[g,P] chi_mu(x_g) chi_nu(x_g), where L L^T is a
    positive-definite Gaussian kernel on naux grid points of a 1-D chain and
    chi are normalised Gaussians centred on nbf chain sites.  The implied
    electron-repulsion tensor is then positive pointwise and positive
    semi-definite, like a real Coulomb operator.
    """
    rng = np.random.default_rng(seed)
    sites = np.arange(nbf, dtype=np.float64) + 0.05 * rng.standard_normal(nbf)
    grid = np.linspace(-2.0, nbf + 1.0, naux)
    v = np.exp(-((grid[:, None] - grid[None, :]) ** 2) / (2 * sigma ** 2))
    w, U = np.linalg.eigh(v)
    w = np.clip(w, 0.0, None)
    L = U * np.sqrt(w)[None, :]                      # v = L L^T
    chi = np.exp(-((grid[:, None] - sites[None, :]) ** 2) / (2 * width ** 2))  # [g][mu]
    # B[P][mu][nu] = sum_g L[g,P] chi[g,mu] chi[g,nu]
    return np.einsum("gP,gm,gn->Pmn", L, chi, chi, optimize=True)


# --------------------------------------------------------------------------
# C, H, occupations, rotations
# --------------------------------------------------------------------------
def make_C(seed: int, nbf: int, norb: int) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 0xC])
    G = rng.standard_normal((nbf, norb))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return np.ascontiguousarray(Q * s[None, :])


def make_H(seed: int, nbf: int) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 0x4])
    A = rng.standard_normal((nbf, nbf))
    H = np.triu(A, 1)
    H = H + H.T
    H[np.diag_indices(nbf)] = rng.uniform(-2.0, 0.0, nbf)
    return H


def make_occupations(seed: int, norb: int, nstrong: int) -> np.ndarray:
    """Strong orbitals first: 1-U(1e-3,5e-2); the rest U(0,2e-2); the weak
    occupations are then rescaled so that the total is nstrong (the number of
    electron pairs).  Rescaling only the weak part keeps every n in [0, 1]
    even when half of the orbitals are strong."""
    rng = np.random.default_rng([int(seed), 0x0])
    n = np.empty(norb)
    n[:nstrong] = 1.0 - rng.uniform(1e-3, 5e-2, nstrong)
    n[nstrong:] = rng.uniform(0.0, 2e-2, norb - nstrong)
    weak = n[nstrong:].sum()
    if norb > nstrong and weak > 0:
        n[nstrong:] *= (nstrong - n[:nstrong].sum()) / weak
    assert np.all(n >= 0.0) and np.all(n <= 1.0)
    return n


def make_antisym(seed: int, it: int, norb: int, scale: float = 1e-2) -> np.ndarray:
    """Antisymmetric generator eps*Y of the small random rotation of iteration ``it``."""
    rng = np.random.default_rng([int(seed), int(it), 0x7])
    Y = rng.standard_normal((norb, norb)) / math.sqrt(norb)
    Y = np.triu(Y, 1)
    return scale * (Y - Y.T)


def make_symmetric(seed: int, norb: int, tag: int = 0x5) -> np.ndarray:
    rng = np.random.default_rng([int(seed), tag])
    A = rng.standard_normal((norb, norb))
    return 0.5 * (A + A.T)


def make_dipoles(seed: int, nbf: int) -> np.ndarray:
    """Three symmetric AO dipole matrices d_x, d_y, d_z with N(0, 0.1) entries."""
    rng = np.random.default_rng([int(seed), 0xD])
    out = np.empty((3, nbf, nbf))
    for a in range(3):
        A = np.triu(rng.normal(0.0, 0.1, (nbf, nbf)))
        out[a] = A + np.triu(A, 1).T
    return out


def field_strengths(h: float = 1e-3, kmax: int = 3):
    """The 25 finite-field instances: zero and +/- h*2^k along x, y, z."""
    fields = [(0, 0.0)]
    for axis in range(3):
        for k in range(kmax + 1):
            for sgn in (+1.0, -1.0):
                fields.append((axis, sgn * h * 2 ** k))
    return fields


def pairing(norb: int, nstrong: int, ng: int):
    """Orbital-pairing structure: for each strong orbital g (0-based), the list
    of its weak partners.  Weak orbitals are assigned in mirrored order, as in
    the pairing figure: the i-th weak orbital of g is nstrong + (nstrong-1-g) +
    i*nstrong.  Orbitals beyond nstrong*(1+ng) belong to no subspace."""
    groups = []
    for g in range(nstrong):
        weak = [nstrong + (nstrong - 1 - g) + i * nstrong for i in range(ng)]
        assert all(w < norb for w in weak)
        groups.append([g] + weak)
    return groups


def field_instances(seed: int, nbf: int, norb: int, nstrong: int, ninst: int = 25,
                    h: float = 1e-3):
    """Finite-field instances sharing one B: the i-th has its own C_i (seeded
    QR), H_i = H + F_i d_axis (base H plus field times a random symmetric
    dipole matrix) and its own occupations.  Fields: 0 and +/- h 2^k, k=0..3,
    along x, y, z (25 instances), truncated to ``ninst``."""
    fields = field_strengths(h)[:ninst]
    H0 = make_H(seed, nbf)
    d = make_dipoles(seed, nbf)
    C = np.stack([make_C(seed + 17 * (i + 1), nbf, norb) for i in range(len(fields))])
    H = np.stack([H0 + F * d[axis] for axis, F in fields])
    n = np.stack([make_occupations(seed + 31 * (i + 1), norb, nstrong) for i in range(len(fields))])
    return dict(C=C, H=H, n=n, fields=fields)
