"""Surrogate network on the GPU against the CPU reference (oracle/mlp.py).

Tolerances: the kernels and the reference round the same values to bfloat16;
they differ by FP32 vs FP64 accumulation, which now and then moves a value
across a bfloat16 rounding boundary (one bfloat16 step, 2^-8 relative, in one
activation or gradient entry).  Predictions are compared by the relative
Frobenius error of each block (C, K, D) with a bound of a few such steps times
the output scales, and the median with a bound far below one step.
"""
import os
import time

import numpy as np
import pytest

import chom_inputs as ci
from gpu_util import banner, require_gpu
from mlp_util import norm_record, rows, weights
from oracle import mlp as ref

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _surrogate(members, seed=0):
    from paper_1610_03484_amd import Surrogate
    return Surrogate(members=members, seed=seed)


def _synthetic_targets(n, seed):
    """Physical-looking outputs: positive diagonal-dominant C, K, D with random variation."""
    u = rows(seed, n, 33, stream=1)
    y_mu = np.concatenate([np.linspace(1.0, 8.0, 21), np.linspace(0.2, 0.6, 6), np.linspace(0.3, 0.9, 6)])
    y = y_mu + 0.2 * y_mu * u
    return y[:, :21].copy(), y[:, 21:27].copy(), y[:, 27:].copy()


def _norm_from(params, C, K, D):
    x_mu, x_sd = ref.column_stats(ref.features(params))
    y_mu, y_sd = ref.column_stats(ref.encode(ref.targets(C, K, D)))
    return x_mu, x_sd, y_mu, y_sd


def _encoded_targets(C, K, D, y_mu, y_sd):
    return ref.standardise(ref.encode(ref.targets(C, K, D)), y_mu, y_sd, quant=False)


@pytest.mark.parametrize("members", [1, 3])
def test_prediction_matches_reference(members):
    require_gpu()
    banner(f"surrogate predict parity, members={members}")
    n = 200                                   # three full workgroups and a ragged one
    params = ci.draw_params(21, n)
    C, K, D = _synthetic_targets(n, 22)
    x_mu, x_sd, y_mu, y_sd = _norm_from(params, C, K, D)
    s = _surrogate(members)
    flats = [weights(30 + m) for m in range(members)]
    for m, f in enumerate(flats):
        s.set_weights(m, f)
    s.set_normalisation(norm_record(x_mu, x_sd, y_mu, y_sd))
    Cg, Kg, Dg, dis = s.predict(params)
    flats32 = [f.astype(np.float32).astype(np.float64) for f in flats]     # what the library holds
    mean, dis_ref = ref.predict(flats32, x_mu, x_sd, y_mu, y_sd, params, quant=True)
    got = np.concatenate([Cg, Kg, Dg], axis=1)
    err = ref.block_errors(got, mean)
    print(f"[mlp] predict members={members}: relative block error max {err.max():.2e}, "
          f"median {np.median(err):.2e}")
    assert err.max() <= 2e-3
    assert np.median(err) <= 1e-4
    if members > 1:
        np.testing.assert_allclose(dis, dis_ref, rtol=2e-2)
        assert dis.min() > 0.0
    else:
        assert np.all(dis == 0.0)
    s.close()


def test_gradient_matches_reference():
    require_gpu()
    banner("surrogate loss gradient parity")
    n = 300                                   # two minibatches of 256, the second ragged
    params = ci.draw_params(23, n)
    C, K, D = _synthetic_targets(n, 24)
    x_mu, x_sd, y_mu, y_sd = _norm_from(params, C, K, D)
    s = _surrogate(2)
    flat = weights(40)
    s.set_weights(1, flat)
    s.set_normalisation(norm_record(x_mu, x_sd, y_mu, y_sd))
    loss, g = s.loss_grad(1, params, C, K, D)
    f32 = flat.astype(np.float32).astype(np.float64)
    xhat = ref.standardise(ref.features(params), x_mu, x_sd, quant=True)
    that = _encoded_targets(C, K, D, y_mu, y_sd)
    loss_ref, g_ref = ref.loss_grad(f32, xhat, that, quant=True)
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    starts = np.cumsum([0] + [o * i + o for i, o in ref.LAYERS])
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    k = 0
    for li, (i, o) in enumerate(ref.LAYERS):
        for part, size in (("W", o * i), ("b", o)):
            a, b = g[k:k + size], g_ref[k:k + size]
            e = np.linalg.norm(a - b) / np.linalg.norm(b)
            print(f"[mlp] grad {names[2 * li + (part == 'b')]}: rel {e:.2e}")
            assert e <= 1e-2, (li, part, e)
            k += size
    assert k == starts[-1]
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) <= 3e-3
    s.close()


def test_adam_step_matches_reference():
    require_gpu()
    banner("surrogate one Adam step parity")
    n = 128
    params = ci.draw_params(25, n)
    C, K, D = _synthetic_targets(n, 26)
    x_mu, x_sd, y_mu, y_sd = _norm_from(params, C, K, D)
    s = _surrogate(1, seed=3)
    flat = weights(41)
    s.set_weights(0, flat)
    s.set_normalisation(norm_record(x_mu, x_sd, y_mu, y_sd))
    lr = 1e-3
    s.train(params, C, K, D, epochs=1, batch=n, lr=lr, lr_final=lr, refit_normalisation=0)
    w1 = s.get_weights(0).astype(np.float64)
    f32 = flat.astype(np.float32).astype(np.float64)
    xhat = ref.standardise(ref.features(params), x_mu, x_sd, quant=True)
    that = _encoded_targets(C, K, D, y_mu, y_sd)
    _, g = ref.loss_grad(f32, xhat, that, quant=True)
    w_ref, _, _ = ref.adam_step(f32, 0 * f32, 0 * f32, g, 1, lr)
    dw, dw_ref = w1 - f32, w_ref - f32
    # the first Adam step is lr * g / (|g| + eps): compare where |g| is clearly non-zero
    big = np.abs(g) > 1e-2 * np.sqrt(np.mean(g * g))
    close = np.abs(dw - dw_ref) <= 1e-3 * lr + 1e-6 * np.abs(f32)
    print(f"[mlp] adam: {big.sum()} clear entries, mismatch fraction {1 - close[big].mean():.2e}")
    assert close[big].mean() >= 0.999
    assert np.all(np.abs(dw) <= lr * 1.001 + 1e-6 * np.abs(f32))
    s.close()


def test_training_reduces_the_loss():
    require_gpu()
    banner("surrogate training reduces the loss")
    n = 2048
    params = ci.draw_params(27, n)
    f = ref.features(params)
    # smooth synthetic map of the features
    basis = np.stack([f[:, 0] / 10, f[:, 1], *(f[:, 2:] - 1.0).T * 10], axis=1)       # [n, 10]
    Wt = rows(28, 10, 33, stream=2)
    y = 2.0 + np.tanh(basis @ Wt) + 0.1 * (basis @ Wt) ** 2
    C, K, D = y[:, :21].copy(), y[:, 21:27].copy(), y[:, 27:].copy()
    s = _surrogate(3, seed=5)
    t0 = time.perf_counter()
    hist = s.train(params, C, K, D, epochs=60, batch=128)
    dt = time.perf_counter() - t0
    print(f"[mlp] 3 members x 60 epochs x {n} rows: {dt:.2f} s, loss {hist[:, 0]} -> {hist[:, -1]}")
    assert np.all(hist[:, -1] < 0.05 * hist[:, 0])
    Cp, Kp, Dp, dis = s.predict(params[:256])
    err = ref.block_errors(np.concatenate([Cp, Kp, Dp], axis=1), y[:256])
    print(f"[mlp] fit error on training rows: median {np.median(err):.2e}, max {err.max():.2e}")
    assert np.median(err) < 2e-2
    assert dis.max() > 0.0
    s.close()


# ---------------------------------------------------------------- surrogate of the RVE solve
HELDOUT = os.path.join(HERE, "golden", "surrogate_heldout_n12_periodic.txt")


def _heldout():
    if not os.path.exists(HELDOUT):
        pytest.skip("held-out oracle file not generated")
    a = np.loadtxt(HELDOUT)
    return a[:, 1:12], a[:, 12:33], a[:, 33:39], a[:, 39:45]


@pytest.fixture(scope="module")
def trained():
    require_gpu()
    from paper_1610_03484_amd import RVE, generate_plain_weave
    banner("surrogate: training set of 12^3 periodic RVE solves")
    mesh = generate_plain_weave(12, device="cuda:0")
    rve = RVE(*mesh, ci.BASE_MATERIALS, bc="periodic", precision="fp32_refined", rtol=1e-10, max_iter=50000)
    ntrain = 8192
    params = ci.draw_params(0, ntrain)
    t0 = time.perf_counter()
    C, K, D = [], [], []
    for s0 in range(0, ntrain, 256):
        c, k, d, _ = rve.homogenise(params[s0:s0 + 256])
        C.append(c)
        K.append(k)
        D.append(d)
        print(f"[mlp] solved {s0 + 256}/{ntrain} training RVEs", flush=True)
    C, K, D = np.concatenate(C), np.concatenate(K), np.concatenate(D)
    t_solve = (time.perf_counter() - t0) / ntrain
    s = _surrogate(5, seed=11)
    t0 = time.perf_counter()
    hist = s.train(params, C, K, D, epochs=200, batch=128)
    t_train = time.perf_counter() - t0
    print(f"[mlp] {t_solve * 1e3:.1f} ms per training solve; training {t_train:.2f} s; "
          f"loss {hist[:, -1]}")
    yield s, rve, t_solve
    s.close()
    rve.close()


def test_surrogate_meets_tolerance_on_heldout_oracle_points(trained):
    s, rve, _ = trained
    p, Cr, Kr, Dr = _heldout()
    C, K, D, dis, used, nfb = s.homogenise(rve, p, thresh=1e-2, chunk=64)
    err = ref.block_errors(np.concatenate([C, K, D], axis=1), np.concatenate([Cr, Kr, Dr], axis=1))
    Cp, Kp, Dp, _ = s.predict(p)
    err_raw = ref.block_errors(np.concatenate([Cp, Kp, Dp], axis=1), np.concatenate([Cr, Kr, Dr], axis=1))
    print(f"[mlp] held-out {len(p)}: network alone max {err_raw.max():.2e} median {np.median(err_raw):.2e}; "
          f"with fallback ({nfb} re-solved) max {err.max():.2e}")
    assert np.all(used[dis > 1e-2] == 1) and np.all(used[dis <= 1e-2] == 0)
    assert nfb == int(used.sum())
    assert err.max() <= 1e-2


def test_surrogate_gain_over_batched_solve(trained):
    s, rve, t_solve = trained
    p = ci.draw_params(2_000_000, 256)
    t0 = time.perf_counter()
    _, _, _, dis, used, nfb = s.homogenise(rve, p, thresh=1e-2, chunk=64)
    t_sur = time.perf_counter() - t0
    t0 = time.perf_counter()
    rve.homogenise(p[:64])
    t_direct = (time.perf_counter() - t0) / 64 * len(p)
    gain = t_direct / t_sur
    print(f"[mlp] 256 points: surrogate+fallback {t_sur * 1e3:.1f} ms ({nfb} fallbacks), "
          f"batched solve {t_direct * 1e3:.1f} ms (from 64), gain x{gain:.1f}")
    assert gain > 1.0
