"""The stored observation series are reproducible from the committed script
(which calls only the oracle), and the workload shapes are as documented."""
import importlib.util
import os

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _maker():
    spec = importlib.util.spec_from_file_location(
        "make_series", os.path.join(ROOT, "synth", "make_series.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_stored_series_regenerate_bitwise(orc):
    m = _maker()
    for name in ("c1", "c2", "c4", "c5", "c3", "paper"):
        fresh = m.MAKERS[name]()
        stored = synth._load(name)
        assert set(fresh) == set(stored)
        for k in fresh:
            np.testing.assert_array_equal(fresh[k], stored[k], err_msg=f"{name}.{k}")


def test_workload_shapes():
    assert synth.c1().particle_steps_per_iter == 256 * 600
    assert synth.c2().particle_steps_per_iter == 8192 * 1800
    c3 = synth.c3()
    assert len(c3.fits) == 512 and all(28 <= f.W <= 365 for f in c3.fits)
    assert all(f.K == -(-f.W // 14) and f.d == f.K + 3 for f in c3.fits)
    assert len({f.stream for f in c3.fits}) == 512
    wl, th = synth.c4()
    assert th.shape == (65536, 16) and wl.fits[0].T == 7300
    assert np.all(th >= wl.fits[0].lo) and np.all(th <= wl.fits[0].hi)
    c5 = synth.c5(windows=[0, 51])
    assert len(c5.fits) == 32 and c5.fits[-1].stream == 16 * 51 + 15
    for f in synth.c1().fits + synth.c2().fits + c3.fits:
        assert f.y.shape == (f.W + 1,) and np.all(np.diff(f.y) >= 0) and f.y[0] == f.D0


def test_paper_shaped_workloads():
    wl = synth.paper()
    f = wl.fits[0]
    assert (f.W, f.spd, f.K, f.n_part, wl.iters, wl.loss) == (92, 1, 4, 10000, 100, "ird_mxse")
    assert (wl.w, wl.c1, wl.c2) == (0.5, 0.5, 0.5)
    o = f.obs3.reshape(3, -1)
    assert o.shape == (3, 93) and tuple(o[:, 0]) == (f.lo[6], f.R0, f.D0)
    assert np.all(np.diff(o[1]) >= 0) and np.all(np.diff(o[2]) >= 0)
    r = synth.rep(n_rep=3)
    assert all(np.array_equal(g.obs3, r.fits[0].obs3) for g in r.fits)
    assert [g.stream for g in r.fits] == [0, 1, 2]


def test_paper_timing_case_matches_the_paper_setup():
    """The paper's swarm settings and timing case (Sec. 3.3), stored in
    tests/golden/pso_setup_sec3_3.txt, are those of the paper workload."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "pso_setup_sec3_3.txt")
    g = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            g[k] = float(v)
    wl = synth.paper()
    (f,) = wl.fits
    assert f.n_part == g["particles"] and wl.iters == g["iterations"]
    assert wl.w == g["inertia"] and wl.c1 == g["cognitive"] and wl.c2 == g["social"]
    assert f.W == g["timing_days"] and wl.loss == "ird_mxse"
    assert f.model == "euler_ramp" and f.spd == 1
