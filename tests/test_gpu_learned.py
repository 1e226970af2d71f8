"""The learned corrector inside the OCI iteration, through the C ABI.

* FP32 inference on the matrix cores against the FP64 oracle network (FP32
  rounding: 1e-4 of the largest output);
* iterate histories (oci_step_history) against the oracle's iterates: the
  same iterates, 1e-11;
* with a corrector whose every correction is rejected, the steps equal the
  plain host-driven steps bit for bit (the accept rule restores the iterate);
* with a corrector trained on the problem's own histories, steps converge to
  the step's exact solution (direct solve) like plain OCI: every accepted
  iterate is a plain OCI iterate judged by the same stopping rule, so at
  tol 1e-13 the error bound tol rho / (1 - rho) is below 1e-11 (rho <= 0.99).
"""
import numpy as np
import pytest

from oracle import balance
from oracle import corrector as ocorr
from oracle import oci as ooci
from oracle.problem import cell_data
from paper_2305_13555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_13555_amd import corrector as C
    from paper_2305_13555_amd import oci
    return torch, oci, C


def rel(a, b):
    return float(np.max(np.abs(a - b))) / float(np.max(np.abs(b)))


@pytest.mark.parametrize("B,J", [(1, 37), (2, 300), (1, 1000)])
def test_forward32_matches_oracle(env, B, J):
    torch, oci, _ = env
    rng = np.random.default_rng(J)
    w = rng.normal(0.0, 0.2, ocorr.num_weights(8, 4))
    x = rng.normal(0.0, 1.0, (B, 8, J))
    with oci.Corrector(8, 4, B, J) as k:
        k.set_weights(w)
        y = k.forward32(torch.from_numpy(x.astype(np.float32)).to("cuda")).cpu().numpy()
    yr, _ = ocorr.forward(w, x, 8, 4)
    assert np.max(np.abs(y - yr)) <= 1e-4 * np.max(np.abs(yr))


@pytest.mark.parametrize("first", [1, 3])
def test_step_history_matches_oracle_iterates(env, first):
    torch, oci, C = env
    p = W.random_small(21, n_angles=8, n_cells=40, n_regions=3, bc=(W.REFLECT, W.VACUUM))
    cd = cell_data(p)
    n = 5
    ref = [ooci.run_oci(p, cd, 1, tol=0.0, max_iters=l)[0]["phi"] for l in range(1, first + n)]
    with oci.OciContext(p, tol=1e-12, max_iters=20000) as ctx:
        phis, conv, info = C.step_history(ctx, n, first)
    assert len(phis) == n
    for i in range(n):
        assert rel(phis[i], ref[first - 1 + i]) < 1e-11, i
    direct = balance.run_direct(p, cd, 1)
    assert rel(conv, direct[0]["phi"]) < 1e-10


def _slab():
    return W.homogeneous_slab(8, 300, 0.99, 0.05, 1.0, n_steps=3)


def test_rejected_corrections_leave_plain_iterates_bit_for_bit(env):
    torch, oci, C = env
    p = _slab()
    w = C.init_weights(8, 4, seed=5) * 50.0   # predictions far off: every correction rejected
    plain, learned = [], []
    with oci.OciContext(p, tol=1e-10, max_iters=50000) as ctx:
        for _ in range(3):
            rc, info, _ = ctx.step_history(0)
            plain.append((ctx.flux().copy(), info))
    with oci.Corrector(8, 4, 1, p.n_cells) as k, \
            oci.OciContext(p, tol=1e-10, max_iters=50000) as ctx:
        k.set_weights(w)
        ctx.set_corrector(k, first=3, period=5)
        for _ in range(3):
            rc, info = ctx.step()
            learned.append((ctx.flux().copy(), info))
        ctx.set_corrector(None)
    for (pp, pi), (lp, li) in zip(plain, learned):
        assert li["corrections"] == 0
        assert li["launches"] > li["iterations"]          # the rejected trials
        assert li["iterations"] == pi["iterations"]
        assert np.array_equal(lp, pp)


def test_trained_corrections_converge_to_the_exact_solution(env):
    torch, oci, C = env
    p = _slab()
    cd = cell_data(p)
    direct = balance.run_direct(p, cd, 3)
    # training data: the first two steps' iterate histories (early and later windows)
    sets = []
    with oci.OciContext(p, tol=1e-12, max_iters=50000) as ctx:
        for first in (1, 40):
            phis, ref, _ = C.step_history(ctx, 16, first)
            x, t, _, _ = C.samples(phis, ref, range(first + 2, first + 16), first)
            sets.append((torch.from_numpy(x).to("cuda"), torch.from_numpy(t).to("cuda")))
    k, hist, _ = C.train_sets(torch, sets, epochs=300, lr=2e-3)
    assert hist[-1] < hist[0]
    infos = []
    with oci.OciContext(p, tol=1e-13, max_iters=50000) as ctx:
        ctx.set_corrector(k, first=3, period=6)
        for s in range(3):
            rc, info = ctx.step()
            assert rc == oci.OCI_OK
            assert rel(ctx.flux(), direct[s]["phi"]) < 1e-10, s
            infos.append(info)
        ctx.set_corrector(None)
    k.close()
    assert sum(i["corrections"] for i in infos) >= 1


def test_set_corrector_rejects_bad_configurations(env):
    torch, oci, C = env
    p = _slab()
    with oci.Corrector(8, 4, 1, 10) as small, oci.Corrector(4, 4, 1, p.n_cells) as wrong, \
            oci.OciContext(p) as ctx:
        for k, first, period in ((small, 3, 4), (wrong, 3, 4)):
            with pytest.raises(oci.OciError):
                ctx.set_corrector(k, first, period)
    with oci.Corrector(8, 4, 1, p.n_cells) as k, oci.OciContext(p) as ctx:
        with pytest.raises(oci.OciError):
            ctx.set_corrector(k, 2, 4)
        with pytest.raises(oci.OciError):
            ctx.set_corrector(k, 3, 0)
    with oci.Corrector(8, 4, 1, p.n_cells) as k, \
            oci.OciContext(p, precision=oci.OCI_PREC_FP32) as ctx:
        with pytest.raises(oci.OciError):
            ctx.set_corrector(k, 3, 4)
