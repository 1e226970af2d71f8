"""GPU parity of the learned corrector's kernels (forward, loss gradient,
Adam) with the FP64 oracle, through the C ABI.

Tolerance: FP64 sums of at most 5 * 64 products per layer over four layers,
in another order than the oracle's: a difference of 1e-12 of the largest
magnitude involved leaves room of about three orders of magnitude."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import corrector as oc  # noqa: E402
from paper_2305_13555_amd import oci  # noqa: E402


def _data(seed, c_in, c_out, B, J, scale=0.25):
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, scale, oc.num_weights(c_in, c_out))
    x = rng.normal(0.0, 1.0, (B, c_in, J))
    t = rng.normal(0.0, 1.0, (B, c_out, J))
    return w, x, t


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _close(got, ref, rtol=1e-12):
    err = np.max(np.abs(got - ref))
    assert err <= rtol * max(np.max(np.abs(ref)), 1e-300), (err, np.max(np.abs(ref)))


# (c_in, c_out, batch, cells): several 256-cell work-groups with a ragged
# tail, meshes shorter than the kernel width, one cell, S_32-sized channels,
# and a layer wider than 64 channels (the untiled weight gradient)
CASES = [(8, 4, 3, 700), (8, 4, 1, 3), (4, 4, 2, 1), (64, 64, 2, 257), (8, 32, 1, 5),
         (128, 8, 2, 90)]


@pytest.mark.parametrize("c_in,c_out,B,J", CASES)
def test_forward_matches_oracle(c_in, c_out, B, J):
    w, x, _ = _data(10 + J, c_in, c_out, B, J)
    with oci.Corrector(c_in, c_out, B, J) as k:
        assert k.num_weights == oc.num_weights(c_in, c_out)
        k.set_weights(w)
        np.testing.assert_array_equal(k.weights(), w)
        y = k.forward(_dev(x))
        torch.cuda.synchronize()
        ref, _ = oc.forward(w, x, c_in, c_out)
        _close(y.cpu().numpy(), ref)


@pytest.mark.parametrize("c_in,c_out,B,J", CASES)
def test_gradient_matches_oracle(c_in, c_out, B, J):
    w, x, t = _data(20 + J, c_in, c_out, B, J)
    with oci.Corrector(c_in, c_out, B, J) as k:
        k.set_weights(w)
        loss, g = k.grad(_dev(x), _dev(t))
    ref_loss, ref_g = oc.grad(w, x, t, c_in, c_out)
    assert loss == pytest.approx(ref_loss, rel=1e-12)
    # per layer, relative to the layer's largest gradient
    k0 = 0
    for s in oc.layer_shapes(c_in, c_out):
        n = int(np.prod(s))
        _close(g[k0:k0 + n], ref_g[k0:k0 + n], rtol=1e-11)
        k0 += n


def test_adam_steps_match_oracle():
    c_in, c_out, B, J = 8, 4, 2, 300
    w, x, t = _data(30, c_in, c_out, B, J)
    xd, td = _dev(x), _dev(t)
    with oci.Corrector(c_in, c_out, B, J) as k:
        k.set_weights(w)
        losses = [k.train_step(xd, td, 1e-3) for _ in range(4)]
        wg = k.weights()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    wr = w.copy()
    ref_losses = []
    for step in range(1, 5):
        L, g = oc.grad(wr, x, t, c_in, c_out)
        ref_losses.append(L)
        wr, m, v = oc.adam(wr, g, m, v, step, 1e-3)
    np.testing.assert_allclose(losses, ref_losses, rtol=1e-11)
    # an update is lr * m_hat / (sqrt(v_hat) + eps): at most ~lr per step, and
    # a weight whose gradient is near zero can turn its small update around
    np.testing.assert_allclose(wg, wr, rtol=0, atol=1e-9)
    assert losses[-1] < losses[0]


def test_positive_homogeneity_is_exact_for_powers_of_two():
    c_in, c_out, B, J = 8, 4, 2, 300
    w, x, _ = _data(40, c_in, c_out, B, J)
    with oci.Corrector(c_in, c_out, B, J) as k:
        k.set_weights(w)
        y1 = k.forward(_dev(x))
        y2 = k.forward(_dev(4.0 * x))
        torch.cuda.synchronize()
    assert torch.equal(y2, 4.0 * y1)


def test_rejects_sizes_beyond_creation():
    with oci.Corrector(8, 4, 2, 100) as k:
        x = torch.zeros((3, 8, 100), dtype=torch.float64, device="cuda")
        with pytest.raises(oci.OciError):
            k.forward(x)
        x = torch.zeros((2, 8, 101), dtype=torch.float64, device="cuda")
        with pytest.raises(oci.OciError):
            k.forward(x)


def test_training_on_solver_histories_lowers_heldout_error():
    """Thin cells, c = 0.99 (hundreds of OCI iterations per step): trained on
    the library's own iterate histories of four steps, the corrector cuts the
    scalar-flux error of the fifth (held-out) step's early iterates by more
    than half (deterministic: seeded weights, fixed reduction order)."""
    from paper_2305_13555_amd import corrector as C
    from paper_2305_13555_amd import workloads
    slab = workloads.homogeneous_slab(16, 2000, 0.99, 0.05, 1.0)
    hist = []
    with oci.OciContext(slab, tol=1e-13, max_iters=100000) as ctx:
        for _ in range(5):
            phis, ref, info = C.step_history(ctx, 16)
            hist.append((phis, ref))
            assert info["iterations"] > 100
            plain = [np.max(np.abs(ref - p)) for p in phis]
            assert all(b < a for a, b in zip(plain, plain[1:]))
    ls = list(range(3, 17))
    xs, ts = zip(*[C.samples(p, r, ls)[:2] for p, r in hist[:4]])
    x = torch.from_numpy(np.concatenate(xs)).to("cuda")
    t = torch.from_numpy(np.concatenate(ts)).to("cuda")
    k, losses, _ = C.train(torch, x, t, epochs=400, lr=2e-3)
    assert losses[-1] < 0.01 * losses[0]
    rows = C.evaluate(torch, k, hist[4][0], hist[4][1], ls)
    k.close()
    assert [r["l"] for r in rows] == ls
    for r in rows:
        assert r["corrected"] < 0.5 * r["plain"], r
