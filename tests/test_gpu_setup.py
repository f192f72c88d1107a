"""GPU set-up: the weighted local extension problems of the first agglomeration step
on the device (amge_kuhn_build with AMGE_BUILD_DEVICE), one workgroup per agglomerate.

The device evaluates the same shared-plan formulation as the host path in another
summation order.  Rounding differences are amplified by the conditioning of the weighted
local problems, which grows with the coefficient contrast r = max(alpha, beta) /
min(alpha, beta); per level A_k and P_k are held to 1e-13 r relative against the host
build and against the oracle (independent local solver), the bar of
tests/test_library_cpu.py.  Per-hex random coefficients make every
agglomerate's problem its own."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _coef(n, seed=5):
    rng = np.random.default_rng(seed)
    return 10 ** rng.uniform(-2, 2, n ** 3), 10 ** rng.uniform(-1, 1, n ** 3)


@pytest.mark.parametrize("kind,n,L", [("curl", 8, 3), ("div", 8, 3), ("curl", 16, 3)])
def test_device_local_problems_match_host_and_oracle(kind, n, L):
    from oracle.hierarchy import build_hierarchy
    from paper_2107_05613_amd import amge
    a, b = _coef(n)
    r = max(a.max(), b.max()) / min(a.min(), b.min())
    dev = amge.build_problem(kind, n, L, a, b, extension="coefficient", device=True)
    hst = amge.build_problem(kind, n, L, a, b, extension="coefficient")
    H = build_hierarchy(kind, n, L, a, b, check_targets=False, extension="coefficient")
    worst_h = worst_o = 0.0
    for k in range(L):
        for i in (0, 2):
            if dev[k][i] is None:
                continue
            Md, Mh, Mo = dev[k][i].to_scipy(), hst[k][i].to_scipy(), (H.A[k] if i == 0 else H.P[k])
            worst_h = max(worst_h, abs(Md - Mh).max() / abs(Mh).max())
            worst_o = max(worst_o, abs(Md - Mo).max() / abs(Mo).max())
    print(f"{kind} n={n}: device vs host {worst_h:.1e}, device vs oracle {worst_o:.1e} (contrast {r:.0e})")
    assert worst_h <= 1e-13 * r
    assert worst_o <= 1e-13 * r


def test_device_set_up_time_64cube_random_coefficients():
    """The 64^3 H(curl) hierarchy with per-hex random alpha (32,768 weighted first-step
    agglomerates): host and device builds agree; their times are printed."""
    from paper_2107_05613_amd import amge
    n = 64
    rng = np.random.default_rng(1)
    a, b = 10 ** rng.uniform(-3, 3, n ** 3), np.ones(n ** 3)
    t0 = time.perf_counter()
    dev = amge.build_problem("curl", n, 5, a, b, extension="coefficient", device=True)
    t1 = time.perf_counter()
    hst = amge.build_problem("curl", n, 5, a, b, extension="coefficient")
    t2 = time.perf_counter()
    r = a.max() / a.min()
    e = max(abs(dev[k][2].to_scipy() - hst[k][2].to_scipy()).max() / abs(hst[k][2].to_scipy()).max()
            for k in range(4))
    print(f"64^3 H(curl), random per-hex alpha: device build {t1 - t0:.2f} s, host build {t2 - t1:.2f} s, "
          f"P difference {e:.1e}")
    assert e <= 1e-13 * r
