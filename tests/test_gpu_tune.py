"""Launch-shape setter and autotuner on the GPU: the shape changes launches,
not results (same steps to rounding, as with OCI_ITERATES_PER_LAUNCH), and
the tuner leaves the context's state where it found it."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2305_13555_amd import oci, tune  # noqa: E402
from paper_2305_13555_amd import workloads as W  # noqa: E402


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _solve(ctx, steps):
    out = torch.zeros((steps, ctx.n_cells, 4), dtype=torch.float64, device="cuda")
    rc, infos = ctx.solve(steps, out)
    assert rc == oci.OCI_OK
    return out.cpu().numpy(), [i["iterations"] for i in infos]


def test_set_iterates_per_launch_changes_launches_not_results():
    p = W.config2(n_steps=6, n_cells=700, n_regions=5, n_angles=32)
    with oci.OciContext(p) as ctx:
        assert ctx.iterates_per_launch == 4
        phi4, it4 = _solve(ctx, 3)
        assert ctx.set_iterates_per_launch(64) == 4        # clamped to what N = 32 allows
        with pytest.raises(oci.OciError):
            ctx.set_iterates_per_launch(0)
        for k in (1, 2, 3):
            assert ctx.set_iterates_per_launch(k) == k
            ctx.set_state(None, 0)
            phik, itk = _solve(ctx, 3)
            for s in range(3):
                assert abs(itk[s] - it4[s]) <= 1
                assert _rel(phik[s], phi4[s]) < 1e-11


def test_shape_is_fixed_for_mixed_precision():
    p = W.config2(n_steps=2, n_cells=300, n_regions=3, n_angles=16)
    with oci.OciContext(p, precision=oci.OCI_PREC_FP32) as ctx:
        assert ctx.set_iterates_per_launch(3) == 1


def test_tune_picks_a_shape_and_restores_the_state():
    p = W.config2(n_steps=10, n_cells=2000, n_regions=8, n_angles=32)
    tune._cache.clear()
    with oci.OciContext(p) as ctx:
        psi0, step0 = ctx.state()
        k, times = tune.tune(ctx, torch, n_steps=4, repeats=2)
        assert sorted(times) == [1, 2, 3, 4] and k == tune.fastest(times)
        assert all(t > 0 for t in times.values())
        assert ctx.iterates_per_launch == k
        psi1, step1 = ctx.state()
        assert step1 == step0 and np.array_equal(psi1, psi0)
        phi_t, _ = _solve(ctx, 3)
        # a second context of the same sizes takes the cached shape
        with oci.OciContext(p) as c2:
            k2, t2 = tune.tune(c2, torch)
            assert k2 == k and t2 == {}
            phi_d, _ = _solve(c2, 3)
    for s in range(3):
        assert _rel(phi_t[s], phi_d[s]) < 1e-11


def test_inner_iterations_setter_and_tuner_for_mixed_precision():
    """The inner iterations per correction change the work between FP64
    iterates, not what a step converges to."""
    p = W.config2(n_steps=6, n_cells=2000, n_regions=8, n_angles=32)
    tune._cache.clear()
    with oci.OciContext(p, precision=oci.OCI_PREC_FP32) as ctx:
        assert ctx.inner_iterations >= 1
        with pytest.raises(oci.OciError):
            ctx.set_inner_iterations(65)
        base, _ = _solve(ctx, 3)
        for m in (1, 3):
            assert ctx.set_inner_iterations(m) == m
            ctx.set_state(None, 0)
            phim, _ = _solve(ctx, 3)
            assert ctx.inner_iterations == m          # fixed: no search
            for s in range(3):
                assert _rel(phim[s], base[s]) < 1e-9
        psi0, step0 = ctx.state()
        m, times = tune.tune(ctx, torch, n_steps=3, repeats=1)
        assert sorted(times) == list(tune.INNER_CANDIDATES) and m == tune.fastest(times)
        assert ctx.inner_iterations == m
        assert ctx.state()[1] == step0
    with oci.OciContext(p) as c64:
        assert c64.inner_iterations == 0 and c64.set_inner_iterations(2) == 0


@pytest.mark.parametrize("precision", [oci.OCI_PREC_FP64, oci.OCI_PREC_FP32], ids=["fp64", "mixed"])
def test_end_fusion_changes_launches_not_results(precision):
    """With the end of step fused or not, a queued solve computes the same
    iterates (same arithmetic, grouped into other launches): the same
    iteration counts and the scalar flux to rounding order; the tuner picks
    one and restores the state."""
    p = W.config2(n_steps=12, n_cells=3000, n_regions=8, n_angles=32)
    tune._cache.clear()
    with oci.OciContext(p, precision=precision) as ctx:
        assert ctx.end_fusion
        if precision == oci.OCI_PREC_FP32:
            ctx.set_inner_iterations(2)   # (no search of the inner count between the solves)
        phi_f, it_f = _solve(ctx, 12)
        assert ctx.set_end_fusion(False) is False and not ctx.end_fusion
        ctx.set_state(None, 0)
        phi_u, it_u = _solve(ctx, 12)
        assert it_u == it_f
        for s in range(12):
            assert _rel(phi_u[s], phi_f[s]) < 1e-12
        psi0, step0 = ctx.state()
        on, times = tune.tune_fusion(ctx, torch, n_steps=3, repeats=1)
        assert sorted(times) == ["fused", "unfused"] and all(t > 0 for t in times.values())
        assert on == (times["fused"] <= times["unfused"]) and ctx.end_fusion == on
        psi1, step1 = ctx.state()
        assert step1 == step0 and np.array_equal(psi1, psi0)
        with oci.OciContext(p, precision=precision) as c2:
            on2, t2 = tune.tune_fusion(c2, torch)
            assert on2 == on and t2 == {} and c2.end_fusion == on
