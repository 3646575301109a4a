"""Pins of the network oracle (oracle/mlp.py): a hand-evaluated forward
pass, gradients against central finite differences, bf16 rounding on
hand-worked bit patterns, and closed forms of the loss and of Adam's first
step.  CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _tiny():
    # F = 2 inputs, H = 2 hidden units, values chosen so that every step can
    # be evaluated by hand
    W1 = [[1.0, -1.0], [0.5, 2.0]]
    b1 = [0.0, -1.0]
    W2 = [[1.0, 1.0], [-1.0, 0.5]]
    b2 = [0.5, 0.0]
    W3 = [2.0, -3.0]
    b3 = 0.25
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]])


def test_forward_by_hand():
    p = _tiny()
    y, h1, h2 = mlp.forward(p, [[1.0, 2.0]], F=2, H=2)
    # pre1 = (1 - 2 + 0, 0.5 + 4 - 1) = (-1, 3.5) -> h1 = (0, 3.5)
    assert h1.tolist() == [[0.0, 3.5]]
    # pre2 = (0 + 3.5 + 0.5, 0 + 1.75 + 0) -> h2 = (4, 1.75)
    assert h2.tolist() == [[4.0, 1.75]]
    # y = 2*4 - 3*1.75 + 0.25
    assert y.tolist() == [3.0]


def test_layout_size():
    F, H = 16, 128
    assert _tiny().size == 2 * 2 + 2 + 2 * 2 + 2 + 2 + 1
    p = np.zeros(H * F + H + H * H + H + H + 1)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, F, H)
    assert W1.shape == (H, F) and W2.shape == (H, H) and W3.shape == (H,)
    assert p.size == 18817


def _fd_grad(p, x, dy, F, H, idx, h=1e-6):
    g = np.zeros(len(idx))
    for n, i in enumerate(idx):
        a = p.copy(); a[i] += h
        b = p.copy(); b[i] -= h
        g[n] = (np.dot(dy, mlp.forward(a, x, F, H)[0]) - np.dot(dy, mlp.forward(b, x, F, H)[0])) / (2 * h)
    return g


def _away_from_kinks(p, x, F, H, margin=1e-3):
    W1, b1, W2, b2, _, _ = mlp.unpack(p, F, H)
    pre1 = x @ W1.T + b1
    h1 = np.maximum(pre1, 0)
    pre2 = h1 @ W2.T + b2
    return np.abs(pre1).min() > margin and np.abs(pre2).min() > margin


@pytest.mark.parametrize("F,H,B", [(5, 8, 7), (3, 4, 1)])
def test_backward_matches_finite_differences_all_params(F, H, B):
    rng = np.random.default_rng(F * 100 + H)
    for _ in range(20):
        p = rng.normal(0, 0.7, H * F + H + H * H + H + H + 1)
        x = rng.normal(0, 1, (B, F))
        if _away_from_kinks(p, x, F, H):
            break
    dy = rng.normal(0, 1, B)
    g = mlp.backward(p, x, dy, F, H)
    fd = _fd_grad(p, x, dy, F, H, range(p.size))
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


def test_backward_full_width_sampled():
    F, H, B = 16, 128, 5
    rng = np.random.default_rng(7)
    p = rng.normal(0, 0.1, H * F + H + H * H + H + H + 1)
    x = rng.uniform(0, 1, (B, F))
    dy = rng.normal(0, 1, B)
    g = mlp.backward(p, x, dy, F, H)
    # a few coordinates in every block of the layout (W1, b1, W2, b2, W3, b3)
    starts = [0, H * F, H * F + H, H * F + H + H * H, H * F + 2 * H + H * H, p.size - 1]
    idx = sorted({min(s + k, p.size - 1) for s in starts for k in (0, 1, 37)})
    fd = _fd_grad(p, x, dy, F, H, idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-8)


def test_inactive_unit_has_zero_gradient():
    p = _tiny()
    # unit 0 of layer 1 is inactive at x = (1, 2): its input weights get no gradient
    g = mlp.backward(p, np.array([[1.0, 2.0]]), np.array([1.0]), F=2, H=2)
    assert g[0] == 0.0 and g[1] == 0.0 and g[4] == 0.0


def _f32(bits):
    return np.array([bits], np.uint32).view(np.float32)


@pytest.mark.parametrize("bits,expect", [
    (0x3F800000, 0x3F800000),   # 1.0 stays
    (0x3F808000, 0x3F800000),   # exactly half an ulp above 1.0: tie, even (down)
    (0x3F818000, 0x3F820000),   # tie with an odd last bit: rounds up
    (0x3F808001, 0x3F810000),   # just above the tie: up
    (0x3F807FFF, 0x3F800000),   # just below the tie: down
    (0xBF808000, 0xBF800000),   # sign does not change the rule
    (0x40490FDB, 0x40490000),   # float32 pi -> bf16 3.140625
    (0x3F7FFFFF, 0x3F800000),   # carry into the exponent
])
def test_bf16_round_bit_patterns(bits, expect):
    got = mlp.bf16_round(_f32(bits)).view(np.uint32)[0]
    assert int(got) == expect


def test_forward_bf16_exact_when_everything_is_representable():
    # small integers and halves are exact in bf16, and so are all the sums
    p = _tiny()
    x = np.array([[1.0, 2.0], [3.0, -1.0]])
    assert np.array_equal(mlp.forward_bf16(p, x, F=2, H=2), mlp.forward(p, x, F=2, H=2)[0])


def test_forward_bf16_rounds_the_weights():
    p = _tiny()
    p[-1] = 1.0 + 2.0 ** -9          # b3 not representable: rounds to 1.0
    y = mlp.forward_bf16(p, np.array([[1.0, 2.0]]), F=2, H=2)
    assert y.tolist() == [2.75 + 1.0]


def test_mse_closed_form():
    loss, g = mlp.mse([1.0, 3.0], [0.0, 1.0])
    assert loss == (1.0 + 4.0) / 2
    assert g.tolist() == [1.0, 2.0]


def test_adam_first_step_moves_by_lr_times_sign():
    # after one step the bias-corrected moments are g and g^2, so (eps -> 0)
    # every parameter moves by exactly lr against the sign of its gradient
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), step=1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
