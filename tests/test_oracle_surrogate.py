"""Pins of the surrogate oracle (MLP, Adam, PCA, gate) against definitions it
does not share code with: brute-force rounding, central finite differences,
closed forms of special cases, constructed low-rank data."""
import numpy as np
import pytest

from oracle import surrogate as OS


def _net(rng, n_in=3, H=5, O=4, scale=0.7):
    _, n = OS.layout(n_in, H, O)
    return rng.normal(0.0, scale, n)


# ---- bfloat16 rounding -------------------------------------------------------


def _bf16_brute(x):
    """Nearest value with the low 16 bits of the float32 pattern zero, found by
    comparing the two bracketing candidates; ties to the even one."""
    out = np.empty_like(x)
    for i, v in enumerate(np.asarray(x, np.float32)):
        u = int(np.array(v).view(np.uint32))
        lo = u & 0xFFFF0000
        hi = lo + 0x10000
        flo = float(np.array(lo, np.uint32).view(np.float32))
        fhi = float(np.array(hi, np.uint32).view(np.float32))
        dl, dh = abs(float(v) - flo), abs(fhi - float(v))
        if dl < dh or (dl == dh and ((lo >> 16) & 1) == 0):
            out[i] = flo
        else:
            out[i] = fhi
    return out


def test_bf16_round_matches_brute_force_and_special_values():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 3000), rng.uniform(-1e-3, 1e-3, 1000)]).astype(np.float32)
    np.testing.assert_array_equal(OS.bf16_round(x), _bf16_brute(x))
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to the even (1.0)
    assert OS.bf16_round(np.array([1.0 + 2.0**-8]))[0] == 1.0
    # 1 + 3 * 2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert OS.bf16_round(np.array([1.0 + 3 * 2.0**-8]))[0] == 1.0 + 2.0**-6
    assert OS.bf16_round(np.array([0.0, -2.0, 0.5]))[1] == -2.0


# ---- activation ----------------------------------------------------------------


def test_silu_special_values_and_derivative():
    assert OS.silu(np.array(0.0)) == 0.0
    assert OS.silu_grad(np.array(0.0)) == 0.5
    z = np.array([40.0, -40.0])
    np.testing.assert_allclose(OS.silu(z), [40.0, 0.0], atol=1e-15)
    zz = np.linspace(-6, 6, 97)
    h = 1e-5
    fd = (OS.silu(zz + h) - OS.silu(zz - h)) / (2 * h)
    np.testing.assert_allclose(OS.silu_grad(zz), fd, rtol=1e-8, atol=1e-10)


# ---- forward / loss / backward -----------------------------------------------


def test_output_is_bias_when_last_weights_are_zero():
    rng = np.random.default_rng(1)
    n_in, H, O = 3, 5, 4
    w = OS.unpack(_net(rng, n_in, H, O), n_in, H, O)
    w["W3"] = np.zeros((H, O))
    p = OS.pack(w, n_in, H, O)
    x = rng.normal(size=(7, n_in))
    y, _ = OS.forward(p, x, n_in, H, O)
    np.testing.assert_array_equal(y, np.broadcast_to(w["b3"], (7, O)))
    # no gradient reaches the hidden layers; dW3 = h2^T dy exactly
    t = rng.normal(size=(7, O))
    _, g = OS.backward(p, x, t, n_in, H, O)
    gd = OS.unpack(g, n_in, H, O)
    for k in ("W1", "b1", "W2", "b2"):
        assert np.all(gd[k] == 0.0)
    np.testing.assert_allclose(gd["b3"], (2.0 / (7 * O)) * (y - t).sum(axis=0), rtol=1e-14)


def test_forward_by_hand_one_unit():
    """n_in = H = O = 1: y = w3 silu(w2 silu(w1 x + b1) + b2) + b3."""
    p = np.array([0.3, -0.2, 1.7, 0.4, -0.9, 0.05])
    x = np.array([[2.0]])
    s = lambda z: z / (1.0 + np.exp(-z))  # noqa: E731
    want = -0.9 * s(1.7 * s(0.3 * 2.0 - 0.2) + 0.4) + 0.05
    y, _ = OS.forward(p, x, 1, 1, 1)
    assert abs(y[0, 0] - want) < 1e-15


def test_loss_is_mean_square():
    assert OS.loss(np.array([[1.0, 2.0], [3.0, 4.0]]), np.array([[0.0, 0.0], [3.0, 6.0]])) == (1 + 4 + 0 + 4) / 4


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    n_in, H, O, B = 3, 5, 4, 6
    p = _net(rng, n_in, H, O)
    x = rng.normal(size=(B, n_in))
    t = rng.normal(size=(B, O))
    _, g = OS.backward(p, x, t, n_in, H, O)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (OS.loss(OS.forward(p + e, x, n_in, H, O)[0], t) - OS.loss(OS.forward(p - e, x, n_in, H, O)[0], t)) / (
            2 * h
        )
    err = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    assert err <= 1e-7, err


def test_bf16_mode_equals_exact_mode_on_representable_values():
    """With every input, weight and intermediate already a bfloat16 value the
    rounding is the identity: both modes agree (checked on a net whose
    activations stay exact: zero first layer, so h1 = silu(b1) rounded)."""
    rng = np.random.default_rng(3)
    n_in, H, O = 2, 4, 3
    w = {k: OS.bf16_round(v) for k, v in OS.unpack(_net(rng, n_in, H, O), n_in, H, O).items()}
    x = OS.bf16_round(rng.normal(size=(5, n_in)))
    p = OS.pack(w, n_in, H, O)
    y0, c0 = OS.forward(p, x, n_in, H, O, bf16=False)
    y1, c1 = OS.forward(p, x, n_in, H, O, bf16=True)
    np.testing.assert_array_equal(c1["a0"], c0["a0"])
    # the difference is only the rounding of the hidden activations
    assert np.max(np.abs(y1 - y0)) <= 2.0**-7 * np.max(np.abs(y0)) * H * 4


# ---- Adam ------------------------------------------------------------------------


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -1e-3, 0.0, 7.5])
    p, m, v = OS.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_constant_gradient_keeps_unit_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves by lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 30):
        p_prev = p
        p, m, v = OS.adam_step(p, g, m, v, t, lr=1e-3)
        np.testing.assert_allclose(p - p_prev, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_adam_descends_a_quadratic():
    p, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 3000):
        p, m, v = OS.adam_step(p, 2.0 * (p - 3.0), m, v, t, lr=0.01)
    assert abs(p[0] - 3.0) < 1e-2


# ---- PCA ---------------------------------------------------------------------------


def test_pca_recovers_a_constructed_low_rank_set():
    """D = mean + C A^T with orthonormal A [P][k] and centred C whose columns
    are orthogonal with known norms: the principal axes span A, the singular
    values are those norms, and projection then reconstruction is exact."""
    rng = np.random.default_rng(4)
    P, k, n = 200, 5, 40
    A, _ = np.linalg.qr(rng.normal(size=(P, k)))
    C0 = rng.normal(size=(n, k))
    C0 -= C0.mean(axis=0)
    Uc, _, _ = np.linalg.svd(C0, full_matrices=False)
    norms = np.array([9.0, 7.0, 5.0, 3.0, 1.0])
    C = Uc * norms
    mean = rng.normal(size=P)
    D = mean + C @ A.T
    m, V, s = OS.pca_fit(D, k)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    np.testing.assert_allclose(s[:k], norms, rtol=1e-10)
    assert np.all(s[k:] < 1e-9)
    np.testing.assert_allclose(V @ V.T, A @ A.T, atol=1e-10)
    np.testing.assert_allclose(m, mean, atol=1e-12)
    rec = OS.pca_reconstruct(OS.pca_project(D, m, V), m, V)
    np.testing.assert_allclose(rec, D, atol=1e-10)


def test_pca_axes_are_covariance_eigenvectors():
    rng = np.random.default_rng(5)
    D = rng.normal(size=(60, 12)) @ rng.normal(size=(12, 12))
    m, V, s = OS.pca_fit(D, 4)
    Cov = (D - m).T @ (D - m)
    for j in range(4):
        np.testing.assert_allclose(Cov @ V[:, j], s[j] ** 2 * V[:, j], rtol=1e-9, atol=1e-9)


# ---- gate ----------------------------------------------------------------------------


def test_gate_two_members_and_threshold_zero():
    rv_mean = np.array([1.0, 2.0, 3.0])
    mem = np.array([[1.0, 2.0, 3.0], [1.0 + 2e-4, 2.0 + 4e-3, 3.0]])
    ok = np.array([True, True, False])
    rv, err, fb = OS.gate(rv_mean, mem, ok, calib=2.0, threshold_kms=1e-3)
    np.testing.assert_allclose(err, 2.0 * np.abs(mem[1] - mem[0]) / np.sqrt(2.0))
    assert fb.tolist() == [0, 1, 1]
    _, _, fb0 = OS.gate(rv_mean, mem, np.ones(3, bool), calib=2.0, threshold_kms=0.0)
    assert fb0.tolist() == [1, 1, 1]


def test_bf16_gradient_stays_close_to_exact_gradient():
    """Rounding operands to bfloat16 (8 significant bits) perturbs the
    gradient by about 2^-8 relative: within 2e-2 in relative L2."""
    rng = np.random.default_rng(6)
    n_in, H, O, B = 5, 32, 16, 64
    p = _net(rng, n_in, H, O, scale=0.3)
    x = rng.normal(size=(B, n_in))
    t = rng.normal(size=(B, O))
    _, g0 = OS.backward(p, x, t, n_in, H, O)
    _, g1 = OS.backward(p, x, t, n_in, H, O, bf16=True)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 2e-2
    assert not np.array_equal(g1, g0)
