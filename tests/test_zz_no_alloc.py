"""The allocation-free network solve (lb_kirchhoff_noalloc, fixed device
scratch) against lb_kirchhoff with a caller workspace (GPU).

Both run the same kernels in the same order on the same beads, so potentials,
node currents and every scalar must agree bit for bit; two calls in a row,
the second on a smaller network, check that the shared scratch carries
nothing from one call to the next.  The first network is also checked
against the FP64 oracle at the network tests' bar."""
import numpy as np
import pytest

from oracle import network as N

pytestmark = pytest.mark.gpu


def _beads(seed, n, box):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box)


def _both(pos, r_c, x_src, x_snk):
    import torch

    from paper_2607_06794_amd.sim import kirchhoff

    t = torch.tensor(pos, dtype=torch.float64, device="cuda:0")
    print(f"[gpu] network no-alloc vs workspace: n={len(pos)} r_c={r_c}", flush=True)
    a = kirchhoff(t, r_c, x_src, x_snk, tol=1e-13)
    b = kirchhoff(t, r_c, x_src, x_snk, tol=1e-13, noalloc=True)
    torch.cuda.synchronize()
    return a, b


def _same(a, b):
    assert np.array_equal(a["V"].cpu().numpy(), b["V"].cpu().numpy())
    assert np.array_equal(a["I"].cpu().numpy(), b["I"].cpu().numpy())
    for k in ("I_tot", "I_ref", "kappa", "rel_residual", "iterations", "edges", "n_source", "n_sink", "max_degree"):
        assert a[k] == b[k], (k, a[k], b[k])


def test_noalloc_matches_workspace_entry_point_twice():
    big = _beads(41, 6000, (60.0, 14.0, 8.0))  # near the noalloc limit of 8192 beads
    a, b = _both(big, 1.6, 8.0, 52.0)
    _same(a, b)
    assert a["edges"] > 6000 and a["iterations"] > 10
    o = N.kirchhoff(big, 1.6, 8.0, 52.0)
    assert a["edges"] == o["edges"]
    assert np.abs(b["V"].cpu().numpy() - o["V"]).max() <= 1e-9
    # second call, smaller network: nothing of the first call may leak in
    small = _beads(42, 700, (30.0, 8.0, 6.0))
    a2, b2 = _both(small, 1.9, 4.0, 26.0)
    _same(a2, b2)
    o2 = N.kirchhoff(small, 1.9, 4.0, 26.0)
    assert a2["edges"] == o2["edges"]
    assert np.abs(b2["V"].cpu().numpy() - o2["V"]).max() <= 1e-9
    assert abs(b2["I_tot"] - o2["I_tot"]) <= 1e-9 * max(1.0, abs(o2["I_tot"]))


def test_noalloc_rejects_oversized_network():
    import torch

    from paper_2607_06794_amd import _lib
    from paper_2607_06794_amd.sim import kirchhoff

    t = torch.zeros((_lib.LB_NET_NOALLOC_MAX_BEADS + 1, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(RuntimeError, match="at most"):
        kirchhoff(t, 2.1, 1.0, 2.0, noalloc=True)
