"""Ensembles (oci_solve_ensemble): one launch per iteration over a work queue of
(problem, tile) entries of many independent problems, against the FP64 oracle.

Each problem keeps its own operators, rings, records and control block, so
its iterates and stopping decisions are those of its own steps: fixed
iteration counts agree with the oracle to 1e-11 (rounding order), converged
steps with the same stopping rule to 1e-10 with iteration counts within one.
The mix has every angle count of the ensemble generator (S8 .. S128), a
slowly converging thin slab (its steps continue alone after the others are
decided) and problems of compact rings.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oci as ooci
from oracle.problem import cell_data
from paper_2305_13555_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2305_13555_amd import oci
    return oci


def rel(a, b):
    return float(np.max(np.abs(a - b))) / float(np.max(np.abs(b)))


def mix(n_steps):
    ps = [dataclasses.replace(W.config5(i), n_steps=n_steps) for i in (7, 57, 9, 5, 2, 30)]
    ps.append(dataclasses.replace(W.homogeneous_slab(8, 300, 0.99, 0.05, 1.0), n_steps=n_steps))
    ps.append(W.layout_case(3, [5, 33, 2, 40], 16, (W.VACUUM, W.INCIDENT)))
    return ps


def run(lib, probs, n_steps, compact=False, caps=None, **kw):
    import torch
    ctxs = [lib.OciContext(p, compact=compact and i % 2 == 0, **kw) for i, p in enumerate(probs)]
    try:
        for c, k in zip(ctxs, caps or []):
            c.set_iterates_per_launch(k)
        outs = [torch.zeros((n_steps, p.n_cells, 4), dtype=torch.float64, device="cuda")
                for p in probs]
        rc, infos = lib.oci_solve_ensemble(ctxs, n_steps, outs)
        return rc, [o.cpu().numpy() for o in outs], infos
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("iters", [1, 3, 6])
def test_ensemble_fixed_iterations_match_oracle(lib, iters):
    probs = mix(2)
    rc, phis, infos = run(lib, probs, 2, tol=0.0, max_iters=iters)
    assert rc == lib.OCI_NOT_CONVERGED
    for p, phi, inf in zip(probs, phis, infos):
        ref = ooci.run_oci(p, cell_data(p), 2, tol=0.0, max_iters=iters)
        for k in range(2):
            assert inf[k]["iterations"] == iters
            assert rel(phi[k], ref[k]["phi"]) < 1e-11, (p.name, k)


def test_ensemble_all_open_after_first_batch_matches_oracle(lib):
    """At most 12 iterations with tol = 0: a fresh step's first batch plans
    8, after which every problem is still open, so the continuation runs over
    the whole set.  Several problems reach a floating-point fixed point after
    9 or more iterations (the change e is exactly 0, which meets tol = 0), in
    the oracle as here, but not at the same iterate: when an iteration stops
    changing in the last bit depends on each side's rounding.  So the counts
    are only bounded (past the first batch, at most the limit) and the scalar
    fluxes, all within rounding of the fixed point, agree with the oracle's."""
    probs = mix(2)
    rc, phis, infos = run(lib, probs, 2, tol=0.0, max_iters=12)
    assert rc == lib.OCI_NOT_CONVERGED
    limited = 0
    for p, phi, inf in zip(probs, phis, infos):
        ref = ooci.run_oci(p, cell_data(p), 2, tol=0.0, max_iters=12)
        for k in range(2):
            assert 9 <= inf[k]["iterations"] <= 12, (p.name, k)
            assert rel(phi[k], ref[k]["phi"]) < 1e-11, (p.name, k)
            limited += inf[k]["iterations"] == 12
    assert limited >= 2


@pytest.mark.parametrize("compact", [False, True])
def test_ensemble_converged_steps_match_oracle(lib, compact):
    probs = mix(3)
    rc, phis, infos = run(lib, probs, 3, compact=compact, tol=1e-10, max_iters=50000)
    assert rc == lib.OCI_OK
    for p, phi, inf in zip(probs, phis, infos):
        ref = ooci.run_oci(p, cell_data(p), 3, tol=1e-10, max_iters=50000)
        for k in range(3):
            assert abs(inf[k]["iterations"] - ref[k]["iterations"]) <= 1, (p.name, k)
            assert rel(phi[k], ref[k]["phi"]) < 1e-10, (p.name, k)
    # the thin slab needs far more iterations than the rest: continued alone
    its = [inf[0]["iterations"] for inf in infos]
    assert max(its) > 10 * min(its)


def same_n_mix(n_steps):
    """Problems of few angle counts, each at several iterate-per-launch caps:
    two S8 slabs (one region), S16 with a 2-cell region (three iterates per
    launch at most), and S16, S32 and S64 ensemble problems."""
    return [dataclasses.replace(W.homogeneous_slab(8, 300, 0.99, 0.05, 1.0), n_steps=n_steps),
            dataclasses.replace(W.homogeneous_slab(8, 77, 0.5, 1.0, 0.1), n_steps=n_steps),
            dataclasses.replace(W.layout_case(3, [5, 33, 2, 40], 16, (W.VACUUM, W.INCIDENT)),
                                n_steps=n_steps),
            dataclasses.replace(W.config5(57), n_steps=n_steps),
            dataclasses.replace(W.config5(9), n_steps=n_steps),
            dataclasses.replace(W.config5(5), n_steps=n_steps)]


@pytest.mark.parametrize("caps", [(4, 1, 3, 4, 3, 4), (1, 4, 4, 2, 4, 1), (3, 3, 1, 3, 4, 3)])
@pytest.mark.parametrize("iters", [2, 5, 7])
def test_ensemble_iterates_per_launch_fixed_match_oracle(lib, caps, iters):
    """Launches of three or four iterates, fewer at the end of a problem's
    range, beside single-iterate problems of the same angle count."""
    probs = same_n_mix(2)
    rc, phis, infos = run(lib, probs, 2, caps=caps, tol=0.0, max_iters=iters)
    assert rc == lib.OCI_NOT_CONVERGED
    for p, phi, inf in zip(probs, phis, infos):
        ref = ooci.run_oci(p, cell_data(p), 2, tol=0.0, max_iters=iters)
        for k in range(2):
            assert inf[k]["iterations"] == ref[k]["iterations"], (p.name, k)
            assert rel(phi[k], ref[k]["phi"]) < 1e-11, (p.name, k)


@pytest.mark.parametrize("caps", [(4, 1, 3, 4, 3, 4), (3, 4, 1, 1, 4, 3)])
def test_ensemble_iterates_per_launch_converged_match_oracle(lib, caps):
    """Converged steps (the slow S8 slab continues in resumed batches of 1,
    1, 2, 4, ... iterates) with the same stopping rule as the oracle."""
    probs = same_n_mix(3)
    rc, phis, infos = run(lib, probs, 3, compact=True, caps=caps, tol=1e-10, max_iters=50000)
    assert rc == lib.OCI_OK
    for p, phi, inf in zip(probs, phis, infos):
        ref = ooci.run_oci(p, cell_data(p), 3, tol=1e-10, max_iters=50000)
        for k in range(3):
            assert abs(inf[k]["iterations"] - ref[k]["iterations"]) <= 1, (p.name, k)
            assert rel(phi[k], ref[k]["phi"]) < 1e-10, (p.name, k)


@pytest.mark.parametrize("tol,iters", [(0.0, 4), (1e-10, 5000)])
def test_ensemble_any_angle_count_matches_oracle(lib, tol, iters):
    """Angle counts without a build of their own (24, 40, 256: the kernels for
    any N, 256 threads per work-group), beside built ones, with every edge
    kind and an initial state, against the oracle."""
    probs = [dataclasses.replace(W.random_small(41, n_angles=24, n_cells=37), n_steps=2),
             dataclasses.replace(W.random_small(42, n_angles=40, n_cells=29,
                                                bc=(W.REFLECT, W.INCIDENT)), n_steps=2),
             dataclasses.replace(W.random_small(43, n_angles=256, n_cells=18), n_steps=2),
             dataclasses.replace(W.random_small(44, n_angles=16, n_cells=33), n_steps=2)]
    rc, phis, infos = run(lib, probs, 2, tol=tol, max_iters=iters)
    assert rc == (lib.OCI_NOT_CONVERGED if tol == 0.0 else lib.OCI_OK)
    for p, phi, inf in zip(probs, phis, infos):
        ref = ooci.run_oci(p, cell_data(p), 2, tol=tol, max_iters=iters)
        for k in range(2):
            if tol == 0.0:
                assert inf[k]["iterations"] == iters
            else:
                assert abs(inf[k]["iterations"] - ref[k]["iterations"]) <= 1, (p.name, k)
            assert rel(phi[k], ref[k]["phi"]) < (1e-11 if tol == 0.0 else 1e-10), (p.name, k)


def test_ensemble_then_ordinary_steps_continue(lib):
    """After an ensemble solve every context continues with its own steps."""
    probs = mix(4)[:3]
    ctxs = [lib.OciContext(p, tol=1e-10) for p in probs]
    try:
        lib.oci_solve_ensemble(ctxs, 2)
        for p, c in zip(probs, ctxs):
            c.step()
            ref = ooci.run_oci(p, cell_data(p), 3, tol=1e-10, max_iters=1000)
            assert rel(c.flux(), ref[2]["phi"]) < 1e-10
            assert c.state()[1] == 3
    finally:
        for c in ctxs:
            c.close()


def test_ensemble_rejects_unsupported_contexts(lib):
    a = lib.OciContext(W.config5(7, n_steps=2))
    odd = lib.OciContext(W.random_small(3, n_angles=6, n_cells=20))
    mixed = lib.OciContext(W.config5(57, n_steps=2), precision=lib.OCI_PREC_FP32)
    b = lib.OciContext(W.config5(9, n_steps=2))
    try:
        for bad in ([a, odd], [a, mixed], [a, a]):
            with pytest.raises(lib.OciError):
                lib.oci_solve_ensemble(bad, 1)
        b.step()   # other step parity
        with pytest.raises(lib.OciError):
            lib.oci_solve_ensemble([a, b], 1)
    finally:
        for c in (a, odd, mixed, b):
            c.close()
