"""Helpers shared by the GPU parity tests (inputs, comparison metrics)."""
import numpy as np
import pytest
import torch

from paper_2512_13550_amd import inputs


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_13550_amd.nof as nof  # noqa: F401  (fails loudly if libnof.so is missing)
    return nof


def dev(x, dtype=torch.float64):
    a = np.ascontiguousarray(x)
    if not a.flags.writeable:          # read-only views (broadcasts) are copied
        a = a.copy()
    return torch.from_numpy(a).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def normwise(a, ref):
    """max|a - ref| / max|ref| (normwise relative error; elementwise relative
    error is meaningless for the many near-zero off-diagonal integrals)."""
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / (den if den > 0 else 1.0))


def case(nbf, naux, norb, seed, decay=8.0):
    B = inputs.make_B(seed, nbf, naux, decay)
    C = inputs.make_C(seed, nbf, norb)
    H = inputs.make_H(seed, nbf)
    n = inputs.make_occupations(seed, norb, max(1, norb // 4))
    cJ = inputs.make_symmetric(seed, norb, 0x11)
    cK = inputs.make_symmetric(seed, norb, 0x12)
    return B, C, H, n, cJ, cK
