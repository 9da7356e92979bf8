"""hlbm_read_coupling_noalloc (the read-out that allocates nothing) against
hlbm_read_coupling, through the C ABI: two calls in a row on lattices of
decreasing size share the one fixed device array, and each must return the
existing entry point's result bit for bit (both run the same kernel in
FP64).  A lattice above the array's capacity is refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(W, H, seed, dims, n, prec):
    sc = W.random_small_scene(seed, dims, n, periodic_z=1, size_range=(1.6, 3.0),
                              gap=-0.8, speed=0.01, spin=0.004)
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=1, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), balance=1, young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, precision=prec)
    g = H.Simulation(p, sc)
    g.init_equilibrium()
    g.step(3)
    return g


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_read_coupling(W, H, prec):
    for seed, dims, n in ((71, (44, 40, 36), 9), (72, (26, 22, 20), 4)):
        _say("no-alloc read-out", dims, n, "precision", prec)
        g = _sim(W, H, seed, dims, n, prec)
        try:
            a = g.coupling()
            b = g.coupling_noalloc()
        finally:
            g.close()
        assert (a["B"] > 0).any() and np.abs(a["up"]).max() > 0
        assert np.array_equal(a["B"], b["B"])
        assert np.array_equal(a["up"], b["up"])


def test_noalloc_refuses_large_lattice(W, H):
    _say("no-alloc read-out above capacity")
    g = _sim(W, H, 73, (160, 128, 128), 3, 1)
    try:
        with pytest.raises(H.HlbmError, match="fixed staging array"):
            g.coupling_noalloc()
        # the context stays usable
        assert g.coupling()["B"].shape == (128, 128, 160)
    finally:
        g.close()
