"""The allocation-free Y = H X (lrei_apply_hamiltonian_noalloc) against the
allocating entry point (lrei_apply_hamiltonian) through the C ABI: two calls
in a row on one GPU, the second on a smaller input, each bitwise equal to the
allocating call (the same kernels and launch shapes) and within 1e-12 of the
oracle's matrix-free product; a request beyond the static scratch is rejected.
"""
import numpy as np
import pytest

from oracle.hamiltonian import apply_H
from workloads import make_config, haar_factor

pytestmark = pytest.mark.gpu


def _case(cfg_id, n, r, seed):
    cfg = make_config(cfg_id, n=n, r=1, with_state=False)
    X = haar_factor(2 ** cfg["n"], r, np.random.default_rng(seed))
    return cfg, X


def test_apply_hamiltonian_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2508_21200_amd import Context
    cases = [_case(3, 16, 16, 1), _case(2, 12, 5, 2)]  # the second is smaller
    ctxs = []
    for cfg, X in cases:
        c = Context(device=0, precision="fp64")
        c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
        ctxs.append(c)
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.full_like(Xd, complex(float("nan"), float("nan")))
        torch.cuda.synchronize()
        c.apply_hamiltonian_noalloc(Xd, Yd)
        c.synchronize()
        Y = Yd.cpu().numpy()
        Y_alloc = c.apply_hamiltonian(X)
        Y_or = apply_H(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"], X)
        print(f"n={cfg['n']} r={X.shape[1]}: max |noalloc - alloc| = {np.abs(Y - Y_alloc).max():.1e}, "
              f"vs oracle {np.abs(Y - Y_or).max() / np.abs(Y_or).max():.1e}")
        assert np.array_equal(Y, Y_alloc)
        assert np.abs(Y - Y_or).max() <= 1e-12 * np.abs(Y_or).max()
    for c in ctxs:
        c.close()


def test_apply_hamiltonian_noalloc_rejects_oversize_input():
    import torch
    from paper_2508_21200_amd import Context, LreiError
    cfg = make_config(2, n=18, r=1, with_state=False)  # N r = 2^18 * 16 > 2^21
    c = Context(device=0, precision="fp64")
    c.set_hamiltonian(cfg["n"], cfg["bonds"], cfg["J"], cfg["h"])
    X = torch.zeros((2 ** 18, 16), dtype=torch.complex128, device="cuda")
    Y = torch.empty_like(X)
    with pytest.raises(LreiError) as ei:
        c.apply_hamiltonian_noalloc(X, Y)
    assert ei.value.status == 1 and "scratch" in str(ei.value)
    c.close()
