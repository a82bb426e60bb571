"""Pins of the learned-apodization oracle: bfloat16 rounding, the convolution against torch,
analytic gradients against central differences, identity networks, the first Adam step."""
import numpy as np
import pytest
import torch

from oracle import apodnet as an


def test_bf16_rounding_ties_to_even_and_matches_torch():
    one = 1.0
    vals = np.array([one, one + 2 ** -8, one + 3 * 2 ** -9, one + 2 ** -7 + 2 ** -8, -2.5e-3, 3.0e38, 1e-40])
    got = an.bf16(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                      # halfway between 1 and 1 + 2^-7: even is 1
    assert got[2] == 1.0 + 2 ** -7            # above halfway
    assert got[3] == 1.0 + 2 ** -6            # halfway, odd lower neighbour: rounds up
    rng = np.random.default_rng(0)
    r = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    want = torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(an.bf16(r), want)


def test_convolution_matches_torch_conv1d():
    rng = np.random.default_rng(1)
    h = rng.standard_normal((3, 7, 20))
    W = rng.standard_normal((5, 7, 5))
    b = rng.standard_normal(5)
    want = torch.nn.functional.conv1d(torch.tensor(h), torch.tensor(W), torch.tensor(b), padding=2).numpy()
    np.testing.assert_allclose(an.conv(h, W, b), want, rtol=0, atol=1e-12)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(2)
    params = {k: v.astype(np.float64) for k, v in an.init_params(3).items()}
    for k in ("b1", "b2", "b3", "b4"):
        params[k] = rng.standard_normal(params[k].shape) * 0.1
    x = rng.standard_normal((4, 16))
    target = rng.standard_normal((4, 16)) * 0.05
    w, cache = an.forward(params, x, bf=False)
    grads = an.backward(params, cache, w, target)
    h = 1e-6
    for k in params:
        flat = params[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = an.loss_fn(an.forward(params, x, bf=False)[0], target)
            flat[i] = old - h
            lm = an.loss_fn(an.forward(params, x, bf=False)[0], target)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            ana = grads[k].reshape(-1)[i]
            assert ana == pytest.approx(num, rel=1e-5, abs=1e-7 * max(1.0, abs(num))), (k, i)


def test_identity_network_passes_positive_inputs():
    """Delta kernels on channel 0 and zero biases: w = relu(normalised x)."""
    p = {k: np.zeros_like(v) for k, v in an.init_params(0).items()}
    p["W1"][0, 0, 2] = 1.0
    p["W2"][0, 0, 2] = 1.0
    p["W3"][0, 0, 2] = 1.0
    p["W4"][0, 0, 2] = 1.0
    rng = np.random.default_rng(4)
    x = rng.standard_normal((5, 128))
    w, _ = an.forward(p, x, bf=False)
    np.testing.assert_allclose(w, np.maximum(an.normalise(x), 0.0), atol=1e-14)


def test_first_adam_step_is_signed_learning_rate():
    p = {"a": np.array([1.0, -2.0, 0.5], np.float32)}
    g = {"a": np.array([0.3, -1e-3, 0.0])}
    opt = an.Adam(p, lr=1e-3)
    p1 = opt.step(p, g)
    want = p["a"] - 1e-3 * g["a"] / (np.abs(g["a"]) + 1e-8)
    np.testing.assert_allclose(p1["a"], want, rtol=1e-6)


def test_training_reduces_the_loss_on_mv_targets():
    from oracle import mv
    rng = np.random.default_rng(5)
    x = rng.standard_normal((64, 128)) + 3.0 * np.cos(0.2 * np.arange(128))[None, :] * rng.standard_normal((64, 1))
    target, _, _ = mv.mv_weights(x)
    params = an.init_params(6)
    opt = an.Adam(params, lr=3e-3)
    losses = []
    for it in range(30):
        w, cache = an.forward(params, x)
        losses.append(an.loss_fn(w, target))
        params = opt.step(params, an.backward(params, cache, w, target))
    assert losses[-1] < 0.5 * losses[0]


def test_fallback_replaces_non_finite_weights():
    x = np.ones((3, 4))
    w = np.full((3, 4), 0.25)
    w[1, 2] = np.nan
    y = an.apply_weights(w, x, fallback=np.array([9.0, 7.0, 5.0]))
    np.testing.assert_allclose(y, [1.0, 7.0, 1.0])


def test_adam_bias_corrections_give_the_learning_rate_for_a_constant_gradient():
    """With the same gradient at every step the bias-corrected moments equal g and g^2 exactly,
    so every step moves each weight by lr * g / (|g| + eps): a missing or wrong correction of
    either moment changes the step size after the first step."""
    p = {"a": np.array([1.0, -2.0, 0.5, 3.0], np.float32)}
    g = {"a": np.array([0.3, -1e-3, 2.0, -40.0])}
    opt = an.Adam(p, lr=1e-3)
    cur = p
    for t in range(1, 6):
        nxt = opt.step(cur, g)
        step = nxt["a"].astype(np.float64) - cur["a"].astype(np.float64)
        np.testing.assert_allclose(step, -1e-3 * np.sign(g["a"]), rtol=2e-3)
        cur = nxt


def _bf16_torch(t):
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_bf16_backward_matches_torch_autograd_with_rounding_at_the_same_points():
    """The bfloat16 network's analytic gradients against torch autograd of the same forward pass:
    layer inputs and weights rounded with straight-through derivatives, and the gradients that
    reach each layer's pre-activation (and the output) rounded by hooks.  A rounding that the
    oracle's backward pass applies at another point, or omits, changes the gradients by about a
    bfloat16 ulp and fails the comparison."""
    F = torch.nn.functional
    rng = np.random.default_rng(8)
    params = an.init_params(9)
    for k in ("b1", "b2", "b3"):
        params[k] = (rng.standard_normal(params[k].shape) * 0.1).astype(np.float32)
    params["b4"] = np.float32([0.01])
    x = rng.standard_normal((6, 32)) * 100.0
    target = rng.standard_normal((6, 32)) * 0.05
    w_ref, cache = an.forward(params, x, bf=True)
    g_ref = an.backward(params, cache, w_ref, target)

    def st(t):  # rounding with a straight-through derivative
        return t + (_bf16_torch(t) - t).detach()

    P = {k: torch.tensor(v.astype(np.float64), requires_grad=True) for k, v in params.items()}
    xt = torch.tensor(x)
    xh = xt / torch.sqrt((xt * xt).mean(dim=1, keepdim=True) + 1e-12)
    a = st(xh)[:, None, :]
    zs = []
    for layer in (1, 2, 3):
        z = F.conv1d(a, st(P[f"W{layer}"]), P[f"b{layer}"], padding=2)
        z.register_hook(_bf16_torch)
        zs.append(z)
        a = st(torch.relu(z))
    out = F.conv1d(a, st(P["W4"]), P["b4"], padding=2)
    out.register_hook(_bf16_torch)
    w = out[:, 0, :]
    M = w.shape[1]
    loss = ((M * w - M * torch.tensor(target)) ** 2).mean()
    loss.backward()
    np.testing.assert_allclose(w.detach().numpy(), w_ref, rtol=1e-12, atol=1e-15)
    for k in params:
        got = P[k].grad.numpy()
        scale = np.abs(g_ref[k]).max()
        assert np.abs(got - g_ref[k]).max() <= 1e-10 * scale, k
