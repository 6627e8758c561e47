"""GPU checks of the proposal network kernels against the float64 reference."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_ref as R  # noqa: E402
from paper_2607_27644_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_27644_amd import rbp as mod
    return mod


def _data(din, dout, B, seed, dens=0.05):
    rng = np.random.default_rng(seed)
    x = (rng.random((B, din)) < dens).astype(np.uint8)
    y = (rng.random((B, dout)) < 0.02).astype(np.uint8)
    lam = rng.uniform(2.0, 9.0, dout).astype(np.float32)
    return x, y, lam


def _dev_bits(bits):
    return torch.from_numpy(W.pack_bits(bits).view(np.int32)).cuda()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("din,h,dout,B", [(64, 512, 160, 300), (576, 512, 1952, 129), (24, 64, 60, 77),
                                          (40, 128, 100, 1000)])
def test_forward_matches_reference(rbp, din, h, dout, B):
    net = rbp.MLP(din, h, dout, seed=5)
    rng = np.random.default_rng(2)
    p = net.get_params().astype(np.float64)
    # non-zero biases to exercise the epilogue
    W1, b1, W2, b2, W3, b3 = R.split(p, din, h, dout)
    b1[:] = rng.normal(0, 0.1, h)
    b2[:] = rng.normal(0, 0.1, h)
    b3[:] = rng.normal(0, 0.5, dout)
    net.set_params(p.astype(np.float32))
    x, _, _ = _data(din, dout, B, 3, dens=0.2)
    got = net.forward(_dev_bits(x)).cpu().numpy()
    ref, _ = R.forward(net.get_params(), x, din, h, dout, mirror=True)
    # same BF16 roundings on both sides; what remains is FP32 vs FP64 accumulation
    # and the rare BF16 rounding decision it flips
    assert rel_err(got, ref) < 5e-3
    assert np.abs(got - ref).max() < 5e-2 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("din,h,dout,B", [(64, 512, 160, 256), (576, 128, 1952, 200)])
def test_gradients_match_reference(rbp, din, h, dout, B):
    net = rbp.MLP(din, h, dout, seed=7)
    x, y, lam = _data(din, dout, B, 4, dens=0.1)
    g, loss = net.gradients(_dev_bits(x), _dev_bits(y), torch.from_numpy(lam).cuda())
    g = g.cpu().numpy()
    lref, gref = R.loss_and_grads(net.get_params(), x, y, lam, din, h, dout, mirror=True)
    assert abs(float(loss.item()) - lref) <= 1e-4 * abs(lref)
    W1, b1, W2, b2, W3, b3 = R.split(g, din, h, dout)
    V1, c1, V2, c2, V3, c3 = R.split(gref, din, h, dout)
    for a, b in [(W1, V1), (b1, c1), (W2, V2), (b2, c2), (W3, V3), (b3, c3)]:
        assert rel_err(a, b) < 1e-2


def test_train_step_is_adam_on_the_gradients(rbp):
    din, h, dout, B = 64, 128, 160, 512
    net = rbp.MLP(din, h, dout, seed=9)
    x, y, lam = _data(din, dout, B, 5)
    xs, ys, ls = _dev_bits(x), _dev_bits(y), torch.from_numpy(lam).cuda()
    p0 = net.get_params().astype(np.float64)
    g, _ = net.gradients(xs, ys, ls)
    net.train_step(xs, ys, ls, lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    want, _, _ = R.adam(p0, g.cpu().numpy().astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    assert np.abs(p1 - want).max() < 1e-6


def test_training_reduces_loss_on_a_learnable_map(rbp):
    """Targets are a fixed function of the inputs (y_j = x_{j mod din}); the loss
    must fall well below its starting value."""
    din, h, dout, B = 64, 256, 160, 1024
    net = rbp.MLP(din, h, dout, seed=11)
    rng = np.random.default_rng(6)
    lam = np.full(dout, 4.0, np.float32)
    ls = torch.from_numpy(lam).cuda()
    loss = torch.zeros(1, device="cuda")
    losses = []
    for step in range(150):
        x = (rng.random((B, din)) < 0.1).astype(np.uint8)
        y = x[:, np.arange(dout) % din]
        net.train_step(_dev_bits(x), _dev_bits(y), ls, lr=2e-3, loss_out=loss)
        losses.append(float(loss.item()))
    assert losses[-1] < 0.2 * losses[0]


def test_forward_chunking_and_empty(rbp):
    net = rbp.MLP(64, 64, 160, seed=1)
    x, _, _ = _data(64, 160, 40000, 8)
    xs = _dev_bits(x)
    full = net.forward(xs).cpu().numpy()
    part = net.forward(xs[17000:17100].contiguous()).cpu().numpy()
    assert np.array_equal(full[17000:17100], part)
    net.forward(xs[:0])


def test_checkpoint_resume_is_exact(rbp, tmp_path):
    """Training split by a save/load (masters, Adam moments and step) equals the
    same training without the split, bit for bit; rbp_mlp_set_params (which
    resets the Adam state) does not."""
    din, h, dout, B = 64, 128, 160, 256
    rng = np.random.default_rng(12)
    lam = torch.from_numpy(rng.uniform(2.0, 9.0, dout).astype(np.float32)).cuda()
    batches = []
    for _ in range(10):
        x = (rng.random((B, din)) < 0.1).astype(np.uint8)
        y = (rng.random((B, dout)) < 0.03).astype(np.uint8)
        batches.append((_dev_bits(x), _dev_bits(y)))
    whole = rbp.MLP(din, h, dout, seed=9)
    for xs, ys in batches:
        whole.train_step(xs, ys, lam, lr=1e-3)
    first = rbp.MLP(din, h, dout, seed=9)
    for xs, ys in batches[:5]:
        first.train_step(xs, ys, lam, lr=1e-3)
    path = str(tmp_path / "net.ckpt")
    first.save(path)
    resumed = rbp.MLP(din, h, dout, seed=123)  # other initial weights, overwritten by the load
    resumed.load(path)
    for xs, ys in batches[5:]:
        resumed.train_step(xs, ys, lam, lr=1e-3)
    assert np.array_equal(resumed.get_params(), whole.get_params())
    reset = rbp.MLP(din, h, dout, seed=123)
    reset.set_params(first.get_params())
    for xs, ys in batches[5:]:
        reset.train_step(xs, ys, lam, lr=1e-3)
    assert not np.array_equal(reset.get_params(), whole.get_params())
    # wrong dimensions and a file that is not a checkpoint are rejected
    with pytest.raises(rbp.RbpError, match="SHAPE"):
        rbp.MLP(din, h, dout + 1, seed=1).load(path)
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint at all")
    with pytest.raises(rbp.RbpError, match="INVALID_ARG"):
        resumed.load(str(bad))


# ---------------------------------------------------------------------------
# Element-wise gradient checks.  Each gradient element is a sum of products
# whose factors carry the rounding errors of the whole forward and backward
# chain.  A running-error bound of the form tau * S holds element by element,
# where S is the same computation carried out over absolute values (so that a
# value obtained by cancellation is charged the error of its terms):
#   forward  F1 = (|x| |W1|^T + |b1|) m1,  F2 = (F1 |W2|^T + |b2|) m2
#            (m1, m2 the ReLU masks)
#   backward A3 = |p - y| / B,  A2 = (A3 |W3|) m2,  A1 = (A2 |W2|) m1
#   S = [A1^T |x|, sum A1, A2^T F1, sum A2, A3^T F2, sum A3]
# An error e in the logit z moves p by at most p (1 - p) e <= |p - y| e, so the
# output gradient has relative error at most e, which is below tau for the
# logits here (|z| <= 30, sums of a few hundred terms).  tau is fixed by the
# arithmetic:
#   FP32 test build: tau = 1e-5 (unit roundoff 6e-8 times sums of at most a
#   few hundred terms per stage);
#   BF16 build: tau = 2^-6.  Both sides round h1, h2, d3, dh2 and dh1 to BF16
#   at the same places; a rounding lands differently only when FP32 and FP64
#   accumulation straddle a rounding boundary, and then moves that factor by
#   one BF16 unit, at most 2^-7 of its value.  Such flips are rare (the
#   accumulation error is about 1e-5 of S, a BF16 unit 2^-8), so an element off
#   by 2^-6 S needs half of its terms flipped the same way (the worst case, all
#   five factors of every term flipped alike, is 5 2^-7).
# Both allow at most 1e-4 of the elements outside the bound: such coincident
# flips, or a ReLU pre-activation within accumulation error of zero that
# switches a whole term on or off on one side only.


def _abs_chain(params, x, y, lam, din, h, dout, mirror):
    """S for every gradient element, in the flat parameter layout (float64)."""
    delta, (xx, h1, h2, W1r, W2r, W3r) = R.forward(params, x, din, h, dout, mirror)
    _, b1, _, b2, _, _ = R.split(np.asarray(params, np.float64), din, h, dout)
    B = xx.shape[0]
    m1, m2 = h1 > 0, h2 > 0
    F1 = (xx @ np.abs(W1r).T + np.abs(b1)) * m1
    F2 = (F1 @ np.abs(W2r).T + np.abs(b2)) * m2
    p = 1.0 / (1.0 + np.exp(np.asarray(lam, np.float64)[None, :] + delta))
    A3 = np.abs(p - np.asarray(y, np.float64)) / B
    A2 = (A3 @ np.abs(W3r)) * m2
    A1 = (A2 @ np.abs(W2r)) * m1
    return np.concatenate([(A1.T @ xx).ravel(), A1.sum(0), (A2.T @ F1).ravel(), A2.sum(0), (A3.T @ F2).ravel(),
                           A3.sum(0)])


def _planted(kind, params, x, y, lam, din, h, dout, mirror):
    """The float64 reference gradient with one planted mistake (CPU only)."""
    _, g = R.loss_and_grads(params, x, y, lam, din, h, dout, mirror)
    g = g.copy()
    delta, (xx, h1, h2, W1r, W2r, W3r) = R.forward(params, x, din, h, dout, mirror)
    B = xx.shape[0]
    z = -(np.asarray(lam, np.float64)[None, :] + delta)
    pr = 1.0 / (1.0 + np.exp(-z))
    rnd = R.bf16 if mirror else (lambda v: v)
    d3r = rnd(-(pr - np.asarray(y, np.float64)) / B)
    dh2r = rnd((d3r @ W3r) * (h2 > 0))
    if kind == "W2_not_transposed":
        dh1 = (dh2r @ W2r.T) * (h1 > 0)
    elif kind == "h1_mask_dropped":
        dh1 = dh2r @ W2r
    else:
        raise ValueError(kind)
    dh1r = rnd(dh1)
    g[:h * din] = (dh1r.T @ xx).ravel()
    g[h * din:h * din + h] = dh1.sum(0)
    return g


def _violations(g, gref, S, tau):
    return int((np.abs(g - gref) > tau * S + 1e-30).sum())


@pytest.mark.parametrize("din,h,dout,B", [(64, 512, 160, 256), (576, 128, 1952, 200), (40, 64, 100, 77)])
def test_fp32_build_gradients_elementwise(rbp, din, h, dout, B):
    """The FP32 test build of the same kernels (FP32 matrix cores) against the
    unrounded float64 reference: gradient elements within 1e-5 S, the loss
    within 1e-5; each planted mistake in the reference is caught."""
    net = rbp.MLP(din, h, dout, seed=7, fp32_test_build=True)
    rng = np.random.default_rng(3)
    p = net.get_params()
    W1, b1, W2, b2, W3, b3 = R.split(p, din, h, dout)
    b1[:] = rng.normal(0, 0.05, h)
    b2[:] = rng.normal(0, 0.05, h)
    b3[:] = rng.normal(0, 0.5, dout)
    net.set_params(p)
    x, y, lam = _data(din, dout, B, 4, dens=0.1)
    g, loss = net.gradients(_dev_bits(x), _dev_bits(y), torch.from_numpy(lam).cuda())
    g = g.cpu().numpy().astype(np.float64)
    params = net.get_params()
    lref, gref = R.loss_and_grads(params, x, y, lam, din, h, dout, mirror=False)
    S = _abs_chain(params, x, y, lam, din, h, dout, mirror=False)
    assert abs(float(loss.item()) - lref) <= 1e-5 * abs(lref)
    ratio = np.abs(g - gref) / (S + 1e-30)
    tau, allowed = 1e-5, max(1, int(1e-4 * g.size))
    base = _violations(g, gref, S, tau)
    print(f"FP32 build: max |g - g_ref| / S = {ratio.max():.3e}, outside 1e-5 S: {base} of {g.size}")
    assert base <= allowed
    for kind in ("W2_not_transposed", "h1_mask_dropped"):
        assert _violations(g, _planted(kind, params, x, y, lam, din, h, dout, False), S, tau) > 10 * allowed, kind
    # one element of the W2 gradient off by 0.1% is one more element outside
    o2 = h * din + h
    i = o2 + int(np.argmax(np.abs(gref[o2:o2 + h * h]) / (S[o2:o2 + h * h] + 1e-30)))
    bad = gref.copy()
    bad[i] *= 1.001
    assert _violations(g, bad, S, tau) == base + 1


@pytest.mark.parametrize("din,h,dout,B", [(64, 512, 160, 256), (576, 128, 1952, 200), (40, 64, 100, 77)])
def test_bf16_gradients_elementwise(rbp, din, h, dout, B):
    """The BF16 product build against the reference that rounds to BF16 at the
    same places: gradient elements within 2^-6 S (at most 1e-4 of them outside);
    the planted mistakes each put far more elements outside."""
    net = rbp.MLP(din, h, dout, seed=7)
    rng = np.random.default_rng(3)
    p = net.get_params()
    W1, b1, W2, b2, W3, b3 = R.split(p, din, h, dout)
    b1[:] = rng.normal(0, 0.05, h)
    b2[:] = rng.normal(0, 0.05, h)
    b3[:] = rng.normal(0, 0.5, dout)
    net.set_params(p)
    x, y, lam = _data(din, dout, B, 4, dens=0.1)
    g, _ = net.gradients(_dev_bits(x), _dev_bits(y), torch.from_numpy(lam).cuda())
    g = g.cpu().numpy().astype(np.float64)
    params = net.get_params()
    _, gref = R.loss_and_grads(params, x, y, lam, din, h, dout, mirror=True)
    S = _abs_chain(params, x, y, lam, din, h, dout, mirror=True)
    tau, allowed = 2.0 ** -6, max(1, int(1e-4 * g.size))
    ratio = np.abs(g - gref) / (S + 1e-30)
    print(f"BF16 build: max |g - g_ref| / S = {ratio.max():.3e}, "
          f"outside 2^-6 S: {_violations(g, gref, S, tau)} of {g.size}")
    assert _violations(g, gref, S, tau) <= allowed
    for kind in ("W2_not_transposed", "h1_mask_dropped"):
        assert _violations(g, _planted(kind, params, x, y, lam, din, h, dout, True), S, tau) > 10 * allowed, kind
