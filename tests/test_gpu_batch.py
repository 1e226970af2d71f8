"""Batched solves (oci_solve_batch) on the GPU through the C ABI: several
independent problems, each context on its own stream, driven concurrently.
Each context runs the same launches as its own oci_solve, so the batch must
reproduce separate solves bit for bit, and converge to the oracle's steps
within the tolerance argument of test_gpu_parity (same rule, FP64)."""
import numpy as np
import pytest

from oracle import oci as ooci
from oracle.problem import cell_data
from paper_2305_13555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_13555_amd import oci
    return oci, torch


SMALL = [
    (0, dict(n_angles=2, n_cells=30, n_regions=2)),
    (1, dict(n_angles=8, n_cells=200, n_regions=3)),
    (2, dict(n_angles=16, n_cells=700, n_regions=4, bc=(W.REFLECT, W.REFLECT))),
    (3, dict(n_angles=12, n_cells=90, n_regions=5, bc=(W.INCIDENT, W.VACUUM))),
]


def problems():
    return [W.random_small(s, **kw) for s, kw in SMALL] + [W.config5(i, n_steps=4)
                                                           for i in (0, 3, 9)]


def test_batch_matches_separate_solves(env):
    oci, torch = env
    steps = 4
    probs = problems()
    ref = []
    for p in probs:
        with oci.OciContext(p) as c:
            out = torch.zeros((steps, p.n_cells, 4), dtype=torch.float64, device="cuda")
            rc, inf = c.solve(steps, out)
            assert rc >= 0
            ref.append((out.cpu().numpy(), [i["iterations"] for i in inf]))
    streams = [torch.cuda.Stream() for _ in probs]
    ctxs = [oci.OciContext(p, stream=s) for p, s in zip(probs, streams)]
    try:
        outs = [torch.zeros((steps, p.n_cells, 4), dtype=torch.float64, device="cuda")
                for p in probs]
        rc, infos = oci.oci_solve_batch(ctxs, steps, outs)
        torch.cuda.synchronize()
        assert rc >= 0
        for k in range(len(probs)):
            assert [i["iterations"] for i in infos[k]] == ref[k][1], k
            assert np.array_equal(outs[k].cpu().numpy(), ref[k][0]), k
    finally:
        for c in ctxs:
            c.close()


def test_batch_matches_oracle_and_host_outputs(env):
    oci, torch = env
    steps = 3
    probs = [W.random_small(s, **kw) for s, kw in SMALL]
    streams = [torch.cuda.Stream() for _ in probs]
    ctxs = [oci.OciContext(p, stream=s) for p, s in zip(probs, streams)]
    try:
        outs = [np.zeros((steps, p.n_cells, 4)) for p in probs]   # host outputs
        rc, infos = oci.oci_solve_batch(ctxs, steps, outs, n_threads=2)
        assert rc == oci.OCI_OK
    finally:
        for c in ctxs:
            c.close()
    for p, out in zip(probs, outs):
        ref = ooci.run_oci(p, cell_data(p), steps, tol=p.tol, max_iters=p.max_iters)
        for k in range(steps):
            s = np.max(np.abs(ref[k]["phi"]))
            assert np.max(np.abs(out[k] - ref[k]["phi"])) / s < 1e-9


def test_batch_rejects_bad_arguments(env):
    oci, torch = env
    p = W.random_small(1, n_angles=4, n_cells=10, n_regions=1)
    with oci.OciContext(p) as c:
        with pytest.raises(oci.OciError) as ei:
            oci.oci_solve_batch([c, c], 1)
        assert ei.value.code == oci.OCI_EINVAL
