"""GPU parity of the warm-start network against its FP64 reference.

The library's network (bf16 matrix-core convolutions, FP32 accumulation and
master weights) is driven through the C ABI; the FP64 NumPy reference
(oracle/cnn.py, pinned by finite differences) evaluates the same parameters
on the same seeded input.

Tolerances.  The GPU stores the input, the convolution weights, every
activation and every activation gradient in bf16 (8 significant bits, unit
roundoff u = 2^-9) and accumulates in FP32.

Forward against the exact FP64 network: a depth-3 network chains about 11
such roundings between input and output, so a relative error of about
sqrt(11) * 2 u ~ 1.3e-2 (RMS) is expected; the bar is 3e-2.

Gradients: the weight gradients are sums over all pixels whose terms cancel
strongly, which multiplies the storage error; against the exact network a
tensor can be off by tens of percent (measured on the CPU with the
bf16-storage reference: up to 0.4).  So the gradients are compared with the
reference that rounds at the same points (store=bf16).  The two then differ
only where the matrix cores' FP32 accumulation and the reference's FP64 sum
round a value to different bf16 neighbours; such a flip changes one stored
value by 2^-8 of itself and its effect spreads through the receptive fields
of the later layers as a compact blob (measured: deviations of 1e-5 to 1e-3
in a few pixels around single points, not along pixel-tile edges, and none
at all in most single-tile cases).  The bars are 2e-3 on the output and 1e-2
per gradient tensor, with 0.98 as the cosine against the exact gradient; one
wrong index, tap or channel gives relative errors of order 1 (a dropped
quarter of the pixels in the weight-gradient sum gave 0.8).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import Oracle, OracleParams, cnn  # noqa: E402
from paper_1807_02137_amd import mgseg, synth  # noqa: E402

M = 4.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def features(rng, B, H, W):
    """Network-input-like values: z in [0, 1], d in [0, 1], a sparse 0/1 mask."""
    x = np.empty((B, 3, H, W))
    x[:, 0] = rng.uniform(0, 1, (B, H, W))
    x[:, 1] = rng.uniform(0, 1, (B, H, W))
    x[:, 2] = (rng.uniform(0, 1, (B, H, W)) < 0.05).astype(float)
    return x


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def groups(base, depth):
    """(name, start, size) of every parameter tensor in the library's order."""
    C, enc, dec = cnn.shapes(base, depth)
    out, off = [], 0
    for tag, lst in (("enc", enc), ("dec", dec)):
        for i, (ic, oc) in enumerate(lst):
            out.append((f"{tag}{i}.w", off, oc * ic * 9)); off += oc * ic * 9
            out.append((f"{tag}{i}.b", off, oc)); off += oc
    out.append(("head.w", off, C[0])); off += C[0]
    out.append(("head.b", off, 1)); off += 1
    return out


CASES = [  # (B, H, W, base, depth, seed): several pixel tiles with ragged edges, one or two 16-channel tiles per block
    (2, 20, 36, 16, 3, 1),
    (1, 32, 32, 16, 4, 2),
    (3, 8, 12, 32, 2, 3),
]
GRAD_CASES = [c + (pw,) for c, pw in zip(CASES, (1.0, 3.5, 0.5))]


@pytest.mark.parametrize("B,H,W,base,depth,seed", CASES)
def test_forward_matches_reference(B, H, W, base, depth, seed):
    say(f"case net forward B{B} {H}x{W} base {base} depth {depth} seed {seed}")
    net = mgseg.Net(base, depth, seed)
    theta, _ = net.params()
    assert theta.size == cnn.param_count(base, depth)
    x = features(np.random.default_rng(seed), B, H, W)
    phi = net.forward(torch.tensor(x, dtype=torch.float32), M).cpu().numpy()
    ref, _ = cnn.forward(theta.astype(np.float64), x, base, depth, M)
    refq, _ = cnn.forward(theta.astype(np.float64), x, base, depth, M, store=cnn.bf16)
    say(f"  rel to exact {rel(phi, ref):.3e}, to bf16-storage ref {rel(phi, refq):.3e}")
    assert rel(phi, ref) <= 3e-2
    assert rel(phi, refq) <= 2e-3
    net.close()


@pytest.mark.parametrize("B,H,W,base,depth,seed,pw", GRAD_CASES)
def test_gradients_match_reference(B, H, W, base, depth, seed, pw):
    say(f"case net gradients B{B} {H}x{W} base {base} depth {depth} seed {seed} pos_weight {pw}")
    net = mgseg.Net(base, depth, seed)
    rng = np.random.default_rng(100 + seed)
    theta, _ = net.params()
    x = features(rng, B, H, W)
    tgt = rng.uniform(-6, 6, (B, H, W))
    net.forward(torch.tensor(x, dtype=torch.float32), M)
    loss = net.backward(torch.tensor(tgt, dtype=torch.float32), M, pw)
    _, g = net.params()
    th = theta.astype(np.float64)
    loss_ref, g_ref = cnn.loss_and_grad(th, x, tgt, base, depth, M, store=cnn.bf16, pos_weight=pw)
    loss_ex, g_ex = cnn.loss_and_grad(th, x, tgt, base, depth, M, pos_weight=pw)
    say(f"  loss {loss:.6f} bf16-storage ref {loss_ref:.6f} exact {loss_ex:.6f}")
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    assert abs(loss - loss_ex) <= 1e-2 * loss_ex
    worst = (0.0, "")
    for name, off, k in groups(base, depth):
        r = rel(g[off:off + k], g_ref[off:off + k])
        worst = max(worst, (r, name))
    cos = float(g @ g_ex / (np.linalg.norm(g) * np.linalg.norm(g_ex)))
    say(f"  worst tensor rel {worst[0]:.3e} ({worst[1]}); cosine to the exact gradient {cos:.6f}")
    assert worst[0] <= 1e-2, worst
    assert cos >= 0.98
    net.close()


def test_adam_steps_follow_the_update_rule():
    say("case net adam")
    base, depth = 16, 3
    net = mgseg.Net(base, depth, 7)
    rng = np.random.default_rng(7)
    x = torch.tensor(features(rng, 2, 16, 16), dtype=torch.float32)
    tgt = torch.tensor(rng.uniform(-6, 6, (2, 16, 16)), dtype=torch.float32)
    m = np.zeros(net.count); v = np.zeros(net.count)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for t in (1, 2, 3):
        net.forward(x, M)
        net.backward(tgt, M)
        p_before, g = net.params()
        g = g.astype(np.float64)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p_before.astype(np.float64) - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        net.adam_step(lr, b1, b2, eps)
        p_after, _ = net.params()
        assert np.abs(p_after - p).max() <= 1e-6 * max(1.0, np.abs(p).max()), t
    net.close()


def test_adam_state_round_trip_resumes_training(tmp_path):
    """A network given another's parameters and Adam state (moments, step
    count) takes the same next step, bit for bit; with the parameters alone
    (moments cleared, bias correction restarted) it does not.  The checkpoint
    of warmstart.save / load carries the same state."""
    say("case net adam state")
    from paper_1807_02137_amd import warmstart
    base, depth = 16, 3
    rng = np.random.default_rng(19)
    x = torch.tensor(features(rng, 2, 24, 40), dtype=torch.float32)
    tgt = torch.tensor(rng.uniform(-6, 6, (2, 24, 40)), dtype=torch.float32)

    def step(n):
        n.forward(x, M)
        n.backward(tgt, M)
        n.adam_step(1e-2)

    a = mgseg.Net(base, depth, 9)
    step(a)
    step(a)
    p, _ = a.params()
    m, v, t = a.adam_state()
    assert t == 2 and np.abs(m).max() > 0 and np.abs(v).max() > 0
    path = str(tmp_path / "ckpt.npz")
    warmstart.save(a, path)
    b = mgseg.Net(base, depth, 123)
    b.set_params(p)
    b.set_adam_state(m, v, t)
    c, _ = warmstart.load(path)
    fresh = mgseg.Net(base, depth, 5)
    fresh.set_params(p)
    assert fresh.adam_state()[2] == 0 and not np.abs(fresh.adam_state()[0]).any()
    for n in (a, b, c, fresh):
        step(n)
    pa = a.params()[0]
    assert np.array_equal(b.params()[0], pa)
    assert np.array_equal(c.params()[0], pa)
    mc, vc, tc = c.adam_state()
    ma, va, ta = a.adam_state()
    assert tc == ta == 3 and np.array_equal(mc, ma) and np.array_equal(vc, va)
    assert not np.array_equal(fresh.params()[0], pa)
    for n in (a, b, c, fresh):
        n.close()


def test_training_lowers_the_loss_on_a_fixed_batch():
    """The loss is a cross-entropy against soft targets q = (1 + t / M) / 2,
    whose minimum over all outputs is the mean binary entropy of q; Adam on
    one batch must remove most of the excess over that minimum."""
    say("case net training")
    net = mgseg.Net(16, 3, 11)
    rng = np.random.default_rng(11)
    xs = features(rng, 4, 32, 32)
    # a target the network can represent: a smooth function of the input
    tgt = M * np.tanh(3.0 * (xs[:, 0] - 0.5) - 2.0 * (xs[:, 1] - 0.5))
    q = np.clip((1.0 + tgt / M) / 2.0, 1e-12, 1 - 1e-12)
    floor = float((-(q * np.log(q) + (1 - q) * np.log(1 - q))).mean())
    x, t = torch.tensor(xs, dtype=torch.float32), torch.tensor(tgt, dtype=torch.float32)
    losses = []
    for _ in range(60):
        net.forward(x, M)
        losses.append(net.backward(t, M))
        net.adam_step(3e-3)
    say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f} (minimum {floor:.4f})")
    assert losses[-1] - floor < 0.3 * (losses[0] - floor)
    net.close()


def test_forward_rejects_bad_shapes():
    for base, depth in ((8, 3), (24, 3), (0, 3), (16, 1), (16, 7), (64, 5)):
        with pytest.raises(mgseg.MgsegError):
            mgseg.Net(base, depth, 0)
    net = mgseg.Net(16, 3, 0)
    with pytest.raises(mgseg.MgsegError):
        net.forward(torch.zeros((1, 3, 18, 16)), M)          # 18 not a multiple of 4
    with pytest.raises(mgseg.MgsegError):
        net.backward(torch.zeros((1, 18, 16)), M)            # no forward yet
    net.close()


def test_context_features_match_the_oracle():
    say("case features seed 1000")
    inst = synth.config1(1000)
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=6))
    o = Oracle(inst.image, inst.markers, OracleParams(levels=6))
    f = s.features().cpu().numpy()
    z, d = o.get("z"), o.get("d")
    assert np.abs(f[0] - z).max() <= 1e-6 * max(1.0, np.abs(z).max())
    assert np.abs(f[1] - d).max() <= 1e-6 * max(1.0, np.abs(d).max())
    mk = np.zeros_like(z)
    for r, c in np.floor(inst.markers).astype(int):
        mk[r, c] = 1.0
    assert np.array_equal(f[2], mk)
    s.close()


def _net_with_head_bias(bias):
    """A network whose output is pushed to one sign everywhere."""
    net = mgseg.Net(16, 3, 5)
    p, _ = net.params()
    p[-1] = bias
    net.set_params(p)
    return net


def test_predicted_phi0_is_taken_when_it_holds_the_markers():
    say("case predict_phi0 accepted seed 1001")
    inst = synth.config1(1001)
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=6))
    net = _net_with_head_bias(50.0)
    phi = net.forward(s.features()[None], M)[0].double().cpu().numpy()
    assert (phi > 0).all()
    assert s.predict_phi0(net)
    assert np.abs(s.get("phi64") - phi).max() <= 1e-6
    assert s.predict_phi0(net, 0.25)
    assert np.abs(s.get("phi64") - 0.25 * phi).max() <= 1e-6
    with pytest.raises(mgseg.MgsegError):
        s.predict_phi0(net, 0.0)
    assert s.stats()["cycles"] == 0
    net.close()
    s.close()


def test_predicted_phi0_that_misses_a_marker_falls_back_to_the_marker_start():
    say("case predict_phi0 rejected seed 1001")
    inst = synth.config1(1001)
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=6))
    phi_setup, res0 = s.get("phi64"), s.stats()["res0"]
    s.solve(1e-6, 60)
    net = _net_with_head_bias(-50.0)
    assert not s.predict_phi0(net)
    assert np.array_equal(s.get("phi64"), phi_setup)
    st = s.stats()
    assert st["cycles"] == 0 and abs(st["res0"] - res0) <= 1e-12 * res0
    net.close()
    s.close()


def test_reset_restores_the_setup_state():
    say("case reset_phi0 seed 1002")
    inst = synth.config1(1002)
    s = mgseg.Solver(inst.image, inst.markers, mgseg.Params(levels=6))
    phi_setup, st0 = s.get("phi64"), s.stats()
    c1 = s.solve(1e-6, 60)
    s.reset_phi0()
    st = s.stats()
    assert np.array_equal(s.get("phi64"), phi_setup)
    assert st["res0"] == st0["res0"] and st["c1"] == st0["c1"] and st["c2"] == st0["c2"]
    c2 = s.solve(1e-6, 60)
    assert c1[0] == c2[0] and c1[1] == c2[1]           # the same solve again, bit for bit
    s.close()


def test_setup_rejects_markers_outside_the_image():
    inst = synth.config1(1000)
    for bad in ([128.0, 5.0], [5.0, -0.5], [5.0, 128.2]):
        mk = np.vstack([inst.markers, bad])
        with pytest.raises(mgseg.MgsegError):
            mgseg.Solver(inst.image, mk, mgseg.Params(levels=6))
