"""The allocation-free ON optimiser (nof_occ_optimize_noalloc: scratch in a
static device array) against nof_occ_optimize with a caller workspace,
through the C ABI: two calls in a row, the second on a smaller problem,
bit-identical iterates, occupations, energies and info."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import dfjk, occupations
from paper_2512_13550_amd import inputs
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def instance(ns, ng, seed):
    norb = ns * (ng + 1)
    B = inputs.make_B(seed, norb, 3 * norb, 8.0)
    C = inputs.make_C(seed, norb, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    hd = np.diag(dfjk.one_electron(inputs.make_H(seed, norb), C)).copy()
    members = occupations.aufbau_members(hd, ns, ng)
    hd[members[:, 0]] -= 1.0
    return norb, members.astype(np.int32), hd, J, K


def run(nof, entry, norb, ns, ng, members, hd, J, K, x0, mapping):
    d = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    mem, hdd, Jd, Kd, g = d(members, torch.int32), d(hd), d(J), d(K), d(x0)
    n = torch.empty(norb, dtype=torch.float64, device="cuda")
    E = torch.empty((), dtype=torch.float64, device="cuda")
    info = torch.zeros(3, dtype=torch.int32, device="cuda")
    p = ctypes.c_void_p
    args = [norb, ns, ng, p(mem.data_ptr()), mapping, nof.FUNC_PNOF5, p(hdd.data_ptr()), 1, p(Jd.data_ptr()),
            p(Kd.data_ptr()), p(g.data_ptr()), p(n.data_ptr()), p(E.data_ptr()), p(info.data_ptr()), 3000, 1e-8]
    stream = p(torch.cuda.current_stream().cuda_stream)
    if entry == "ws":
        ws = torch.empty(nof.lib.nof_occ_ws(norb, ns, ng), dtype=torch.uint8, device="cuda")
        rc = nof.lib.nof_occ_optimize(*args, p(ws.data_ptr()), ws.numel(), stream)
    else:
        rc = nof.lib.nof_occ_optimize_noalloc(*args, stream)
    torch.cuda.synchronize()
    assert rc == 0, nof.lib.nof_status_str(rc)
    return g.cpu().numpy(), n.cpu().numpy(), float(E), info.cpu().numpy()


@pytest.mark.parametrize("mapping", [0, 1])
def test_noalloc_matches_workspace_entry(mapping):
    nof = need_gpu()
    for ns, ng, seed in ((60, 3, 1), (12, 2, 2)):          # second call smaller than the first
        norb, members, hd, J, K = instance(ns, ng, seed)
        x0 = np.full((ns, ng), 0.3 if mapping == 0 else -3.0)
        print(f"case noalloc map={mapping} norb={norb} ns={ns} ng={ng}", flush=True)
        a = run(nof, "ws", norb, ns, ng, members, hd, J, K, x0, mapping)
        b = run(nof, "noalloc", norb, ns, ng, members, hd, J, K, x0, mapping)
        assert a[3][1] == 1 and a[3][2] == 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert a[2] == b[2] and np.array_equal(a[3], b[3])


def test_noalloc_rejects_problems_beyond_its_scratch():
    nof = need_gpu()
    # 3000 orbitals: M alone is 72 MB, beyond the 32 MiB static scratch
    assert nof.lib.nof_occ_ws(3000, 100, 1) > 32 << 20
    f = ctypes.c_void_p(4096)
    rc = nof.lib.nof_occ_optimize_noalloc(3000, 100, 1, f, 0, 1, f, 1, f, f, f, None, None, None, 10, 1e-8, None)
    assert rc == nof.E_DIM
