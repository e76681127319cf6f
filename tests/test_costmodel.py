"""The benchmark's ALU cost table equals what the ISA probe measures on the
library's own gfx950 build (hipcc cross-compiles here; no GPU needed)."""
import shutil

import pytest


@pytest.mark.skipif(shutil.which("hipcc") is None and not __import__("os").path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_cost_table_matches_isa_probe():
    import bench
    from paper_2403_08692_amd.costmodel import isa_costs

    measured = isa_costs.measure()
    for k, v in bench.COST.items():
        assert measured[k] == v, (k, measured[k], v)
    measured64 = isa_costs.measure(fp64=True)
    for k, v in bench.COST_F64.items():
        assert measured64[k] == v, (k, measured64[k], v)
        assert v <= bench.COST[k]


def test_algorithmic_ops_scale():
    import bench

    # one LEP-like event: 123 active ends (63 quark, 60 gluon), 31 cycles, 3 emissions
    ops = bench.algorithmic_ops(1, 123, 63 + 6 * 60, 31, 3)
    assert 3e4 < ops < 1.5e5
    # work is additive over events
    assert bench.algorithmic_ops(2, 246, 2 * 423, 62, 6) == pytest.approx(2 * ops)


def test_shape_chi2_detects_a_biased_cut():
    import numpy as np

    import bench

    rng = np.random.default_rng(3)
    a, b = rng.normal(size=200_000), rng.normal(size=150_000)

    def h(x):
        return np.histogram(x, bins=50, range=(-3, 3))[0].astype(float)

    assert 0.4 < bench.shape_chi2(h(a), h(b)) < 1.7  # same distribution (49 ndf: 1 +- 0.2)
    assert bench.shape_chi2(h(a[np.abs(a) < 2.5]), h(b)) > 20  # tails cut away
