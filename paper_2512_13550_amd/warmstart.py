"""Learned warm start of the occupation optimiser: training data from the
plain optimiser, training on the GPU with the library's own forward/backward
and ADAM kernels, and the warm- versus cold-start comparison.

Synthetic ON instances (stand-ins for molecules): B, C, H from the seeded
generators, J, K, h from the library's transform; orbital roles by ascending
h_pp (aufbau): the ns lowest orbitals are strong, paired with N_g =
(norb - ns) // ns weak ones in the mirrored order; the strong orbitals' h_pp is
lowered by `gap` (the occupied-virtual gap a molecule has and random matrices
lack).  The optimiser is the library's L-BFGS (softmax map for the training
data; either map in the evaluation).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from paper_2512_13550_amd import inputs


def aufbau_members(hdiag: np.ndarray, ns: int, ng: int) -> np.ndarray:
    order = np.argsort(hdiag, kind="stable")
    members = np.zeros((ns, ng + 1), dtype=np.int32)
    for g in range(ns):
        members[g, 0] = order[g]
        for i in range(ng):
            members[g, 1 + i] = order[ns + (ns - 1 - g) + i * ns]
    return members


class InstanceFactory:
    """Seeded ON instances of a given size sharing one B per basis size."""

    def __init__(self, nof, device="cuda", naux_factor=4, decay=25.0, gap=0.5, bseed=4000):
        self.nof, self.dev = nof, torch.device(device)
        self.naux_factor, self.decay, self.gap, self.bseed = naux_factor, decay, gap, bseed
        self._B = {}

    def B(self, nbf):
        if nbf not in self._B:
            B = inputs.make_B(self.bseed + nbf, nbf, self.naux_factor * nbf, self.decay, threads=16)
            self._B[nbf] = torch.from_numpy(B).to(self.dev)
        return self._B[nbf]

    def make(self, seed, nbf, ns, mapping=1):
        nof = self.nof
        norb = nbf
        ng = max(1, (norb - ns) // ns)
        C = torch.from_numpy(inputs.make_C(seed, nbf, norb)).to(self.dev)
        H = torch.from_numpy(inputs.make_H(seed, nbf)).to(self.dev)
        b, D = nof.mo_transform(self.B(nbf), C)
        h = nof.one_electron(H, C)
        J, K = nof.jk_diag(b, D)
        del b, D
        hd = torch.diagonal(h).contiguous()
        members = aufbau_members(hd.cpu().numpy(), ns, ng)
        shift = torch.zeros(norb, dtype=torch.float64, device=self.dev)
        shift[torch.from_numpy(members[:, 0].astype(np.int64)).to(self.dev)] = -self.gap
        hd = hd + shift
        occ = nof.Occupations(norb, torch.from_numpy(members).to(self.dev), mapping, nof.FUNC_PNOF5)
        return dict(norb=norb, ns=ns, ng=ng, h=hd, J=J, K=K, members=members, occ=occ, mapping=mapping,
                    nof=nof)


def cold_gamma(inst, nstrong=0.98):
    """n_g = 0.98 with the hole shared equally among the weak orbitals, for
    either map: the occupations are handed to the device-side map inversion
    (nof_mlp_warm_gamma) as the angles theta with cos^2 theta = n."""
    nof = inst["nof"]
    ng, norb = inst["ng"], inst["norb"]
    dev = inst["h"].device
    members = torch.from_numpy(inst["members"]).to(dev)
    theta = torch.full((norb,), 0.5 * math.pi, dtype=torch.float32, device=dev)      # n = 0
    theta[members[:, 1:].reshape(-1).long()] = math.acos(math.sqrt((1.0 - nstrong) / ng))
    theta[members[:, 0].long()] = math.acos(math.sqrt(nstrong))
    return nof.mlp_warm_gamma(theta, members, inst["mapping"], norb, 0.0)


def solve(inst, gamma0, maxit=3000, tol=1e-8):
    g = gamma0.clone()
    E, n, info = inst["occ"].optimize(g, inst["h"], inst["J"], inst["K"], maxit=maxit, tol=tol)
    info = info.cpu().numpy()
    return float(E), n, int(info[0]), bool(info[1]), g


def build_dataset(nof, factory, seeds, sizes, ns_range, rng, log=None):
    """Features and target angles of the converged ONs of each instance."""
    Xs, Ts, iters = [], [], []
    for k, s in enumerate(seeds):
        if log and k % 500 == 0:
            log(f"instance {k}")
        nbf = int(rng.choice(sizes))
        ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
        inst = factory.make(int(s), nbf, ns)
        E, n, it, ok, _ = solve(inst, cold_gamma(inst))
        Xs.append(nof.mlp_features(inst["h"], inst["J"], inst["K"]))
        Ts.append(nof.mlp_targets(n))
        iters.append(it)
    return torch.cat(Xs), torch.cat(Ts), np.array(iters)


def init_params(nof, seed, device):
    """Glorot-uniform weights, zero biases (same recipe as the reference network)."""
    rng = np.random.default_rng([seed, 0x3A])
    parts = []
    for name, shp in [("W1", (5, 128)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
                      ("w3", (128,)), ("b3", (1,))]:
        k = int(np.prod(shp))
        if name.startswith("b"):
            parts.append(np.zeros(k))
        else:
            a = math.sqrt(6.0 / (shp[0] + (shp[1] if len(shp) > 1 else 1)))
            parts.append(rng.uniform(-a, a, k))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == nof.lib.nof_mlp_nparams()
    return torch.from_numpy(p).to(device)


def train(nof, X, T, epochs=40, batch=4096, lr=2e-3, seed=0, log=None):
    dev = X.device
    params = init_params(nof, seed, dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.empty_like(params)
    loss = torch.empty((), dtype=torch.float32, device=dev)
    ws = nof.workspace(nof.lib.nof_mlp_ws(batch), dev)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    rows = X.shape[0]
    t = 0
    history = []
    for ep in range(epochs):
        perm = torch.randperm(rows, generator=gen).to(dev)
        tot = 0.0
        for lo in range(0, rows, batch):
            idx = perm[lo:lo + batch]
            xb, tb = X[idx].contiguous(), T[idx].contiguous()
            nof.mlp_loss_grad(xb, tb, params, grad, loss, ws)
            t += 1
            nof.mlp_adam(params, grad, m, v, t, lr=lr)
            tot += float(loss) * idx.numel()
        history.append(tot / rows)
        if log:
            log(f"epoch {ep} loss {history[-1]:.3e}")
    return params, history


WARM_FLOOR = 1e-3   # smallest occupation share of a warm start (see warm_gamma)


def warm_gamma(nof, inst, params, nfloor=WARM_FLOOR):
    """Variables of the optimiser from the network's angles.  Shares below
    nfloor are raised to it: the softmax variable of a near-empty weak orbital
    sits where its gradient (proportional to n) vanishes, so a coarse
    prediction of a tiny occupation would start the optimiser on a plateau."""
    X = nof.mlp_features(inst["h"], inst["J"], inst["K"])
    theta = nof.mlp_forward(X, params)
    members = torch.from_numpy(inst["members"]).to(X.device)
    return nof.mlp_warm_gamma(theta, members, inst["mapping"], inst["norb"], nfloor)


def evaluate(nof, factory, params, seeds, nbf, ns, mapping=1):
    """Iterations and converged energies from the cold start, the network's
    warm start, and (as the ideal reference) a restart from the converged
    variables themselves, with the optimiser on the given map (1 softmax,
    0 trigonometric)."""
    rows = []
    for s in seeds:
        inst = factory.make(int(s), nbf, ns, mapping=mapping)
        Ec, _, ic, okc, gc = solve(inst, cold_gamma(inst))
        Ew, _, iw, okw, _ = solve(inst, warm_gamma(nof, inst, params))
        _, _, ir, _, _ = solve(inst, gc)
        rows.append(dict(seed=int(s), iters_cold=ic, iters_warm=iw, iters_restart=ir, E_cold=Ec,
                         E_warm=Ew, converged=bool(okc and okw)))
    return rows
