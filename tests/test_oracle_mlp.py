"""Pins of the surrogate network's CPU reference (oracle/mlp.py)."""
import math

import numpy as np
import pytest
import torch

import chom_inputs as ci
from mlp_util import rows as _rows
from mlp_util import weights as _weights
from oracle import materials as mats
from oracle import mlp


def test_param_count_and_layout():
    assert mlp.n_params() == 10 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 36 + 36 == 143652
    flat = np.arange(mlp.n_params(), dtype=float)
    Wb = mlp.unpack(flat)
    assert Wb[0][0].shape == (256, 10) and Wb[0][0][0, 1] == 1.0 and Wb[0][1][0] == 2560.0
    assert Wb[3][0].shape == (36, 256) and Wb[3][1][-1] == mlp.n_params() - 1
    np.testing.assert_array_equal(mlp.pack(Wb), flat)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-30, 30, 4000),
                        [0.0, -0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e-39, 65504.0]])
    # exact ties of FP32 values half-way between two bfloat16 values
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64)
    x = np.concatenate([x, ties, -ties])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # GELU(1) = Phi(1), Phi(1) = 0.8413447460685429
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-1.0]))[0] + (1 - 0.8413447460685429)) < 1e-15
    z = np.linspace(-6, 6, 241)
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-9)
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_features_follow_degradation_law():
    p = ci.draw_params(11, 64)
    f = mlp.features(p, c_sat=1.5)
    keep = mats.stiffness_factor(p[:, 0], p[:, 1], p[:, 2], 1.5)
    np.testing.assert_allclose(np.exp(f[:, 0]), keep, rtol=1e-14)
    np.testing.assert_allclose(f[:, 1], keep, rtol=1e-14)
    np.testing.assert_array_equal(f[:, 2:], p[:, 3:])
    # no exposure -> no degradation
    p0 = p.copy()
    p0[:, 2] = 0.0
    assert np.all(mlp.features(p0)[:, 0] == 0.0)


def test_gradient_matches_finite_differences():
    flat = _weights(5)
    x = _rows(6, 5, mlp.N_FEAT)
    t = _rows(7, 5, mlp.N_OUT)
    loss, g = mlp.loss_grad(flat, x, t, quant=False)
    y, _ = mlp.forward(flat, x, quant=False)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-15
    # sample parameters from every tensor of the flat layout
    starts = np.cumsum([0] + [o * i + o for i, o in mlp.LAYERS])
    idx = []
    rng = np.random.default_rng(0)
    for li, (i, o) in enumerate(mlp.LAYERS):
        s = starts[li]
        idx += list(s + rng.integers(0, o * i, 6)) + list(s + o * i + rng.integers(0, o, 3))
    h = 1e-6
    for k in idx:
        fp = flat.copy()
        fp[k] += h
        fm = flat.copy()
        fm[k] -= h
        fd = (mlp.loss_grad(fp, x, t, quant=False)[0] - mlp.loss_grad(fm, x, t, quant=False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g).max()), (k, fd, g[k])


def test_planted_backward_mistake_is_caught(monkeypatch):
    flat = _weights(5)
    x = _rows(6, 3, mlp.N_FEAT)
    t = _rows(7, 3, mlp.N_OUT)
    monkeypatch.setattr(mlp, "gelu_grad", lambda z: 0.5 * (1.0 + np.tanh(z)))   # wrong derivative
    _, g = mlp.loss_grad(flat, x, t, quant=False)
    k = 2560 + 256 + 5                       # an entry of W2
    h = 1e-6
    fp = flat.copy()
    fp[k] += h
    fm = flat.copy()
    fm[k] -= h
    monkeypatch.undo()
    fd = (mlp.loss_grad(fp, x, t, quant=False)[0] - mlp.loss_grad(fm, x, t, quant=False)[0]) / (2 * h)
    assert abs(fd - g[k]) > 1e-6 * abs(fd)


def test_quantised_pass_stays_within_bf16_error():
    flat = _weights(8)
    x = _rows(9, 16, mlp.N_FEAT)
    yq, _ = mlp.forward(flat, mlp.bf16(x), quant=True)
    yf, _ = mlp.forward(flat, x, quant=False)
    scale = np.abs(yf).max()
    assert np.abs(yq - yf).max() <= 0.05 * scale
    assert np.abs(yq - yf).max() > 0.0


def test_adam_closed_form_first_steps():
    rng = np.random.default_rng(1)
    w0 = rng.standard_normal(50)
    g1 = rng.standard_normal(50)
    lr = 1e-3
    w1, m1, v1 = mlp.adam_step(w0, 0 * w0, 0 * w0, g1, 1, lr)
    np.testing.assert_allclose(w1, w0 - lr * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-15)
    g2 = rng.standard_normal(50)
    w2, _, _ = mlp.adam_step(w1, m1, v1, g2, 2, lr)
    m = 0.1 * 0.9 * g1 + 0.1 * g2
    v = 0.001 * 0.999 * g1 ** 2 + 0.001 * g2 ** 2
    mh, vh = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    np.testing.assert_allclose(w2, w1 - lr * mh / (np.sqrt(vh) + 1e-8), rtol=1e-13)


def test_encoding_round_trip_and_scale_invariance():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((9, 33)) + 3.0
    T = mlp.encode(Y)
    assert T.shape == (9, 36)
    np.testing.assert_allclose(mlp.decode(T), Y, rtol=1e-14)
    # scaling a block moves only its log-norm column
    Y2 = Y.copy()
    Y2[:, :21] *= 7.0
    T2 = mlp.encode(Y2)
    np.testing.assert_allclose(T2[:, 0], T[:, 0] + np.log(7.0), rtol=1e-14)
    np.testing.assert_allclose(T2[:, 1:], T[:, 1:], rtol=1e-13)
    # decoding renormalises the direction: scaling it changes nothing
    T3 = T.copy()
    T3[:, 1:22] *= 1.3
    np.testing.assert_allclose(mlp.decode(T3), Y, rtol=1e-14)
    # unit C block: ||C||_F = sqrt(6) for the identity
    eye = np.zeros((1, 33))
    eye[0, [0, 6, 11, 15, 18, 20]] = 1.0
    eye[0, 21:24] = 1.0
    eye[0, 27:30] = 1.0
    assert abs(mlp.encode(eye)[0, 0] - 0.5 * math.log(6.0)) < 1e-15


def test_ensemble_mean_and_disagreement():
    p = ci.draw_params(12, 7)
    zeros = np.zeros(mlp.n_params())
    mu = np.zeros(10)
    sd = np.ones(10)
    phys = np.linspace(1.0, 3.0, 33)
    enc = mlp.encode(phys[None, :])[0]
    # zero weights: the output is the last bias, whatever the input
    b_a = zeros.copy()
    b_a[-36:] = 0.0
    y_sd = np.full(36, 0.01)
    mean, dis = mlp.predict([b_a, b_a], mu, sd, enc, y_sd, p)
    np.testing.assert_allclose(mean, np.tile(phys, (7, 1)), rtol=1e-13)
    assert np.all(dis == 0.0)
    # two members whose log-norm outputs differ by +-h: the blocks scale by exp(+-h*0.01)
    h = 1.0
    b_p, b_m = zeros.copy(), zeros.copy()
    for k in (0, 22, 29):
        b_p[-36 + k] = h
        b_m[-36 + k] = -h
    mean, dis = mlp.predict([b_p, b_m], mu, sd, enc, y_sd, p)
    s = 0.01 * h
    np.testing.assert_allclose(mean, np.tile(phys * math.cosh(s), (7, 1)), rtol=1e-13)
    # sample std of {e^s, e^-s} x is sqrt(2)|sinh(s)| x; relative to the mean cosh(s) x
    np.testing.assert_allclose(dis, math.sqrt(2.0) * math.sinh(s) / math.cosh(s), rtol=1e-10)


def test_block_errors_closed_form():
    ref = np.ones((1, 33))
    pred = ref.copy()
    pred[0, 0] += 0.5                      # C_11 only: ||dC||_F = 0.5, ||C||_F = 6 (36 unit entries)
    assert abs(mlp.block_errors(pred, ref)[0] - 0.5 / 6.0) < 1e-15
    pred = ref.copy()
    pred[0, 21 + 3] += 0.3                 # K_xy: counted twice
    assert abs(mlp.block_errors(pred, ref)[0] - math.sqrt(2 * 0.09) / 3.0) < 1e-15


def test_heldout_file_matches_its_seeded_records():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "surrogate_heldout_n12_periodic.txt")
    a = np.loadtxt(path)
    assert a.shape == (256, 45)
    np.testing.assert_array_equal(a[:, 0], np.arange(256))
    np.testing.assert_array_equal(a[:, 1:12], ci.draw_params(1_000_000, 256))
    # C_bar symmetric positive definite, K_bar and D_bar positive diagonals
    iu = np.triu_indices(6)
    Cm = np.zeros((256, 6, 6))
    Cm[:, iu[0], iu[1]] = a[:, 12:33]
    Cm[:, iu[1], iu[0]] = a[:, 12:33]
    assert np.all(np.linalg.eigvalsh(Cm) > 0)
    assert np.all(a[:, 33:36] > 0) and np.all(a[:, 39:42] > 0)
