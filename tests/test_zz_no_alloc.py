"""chom_mlp_loss_grad_noalloc (static workspace, no allocation) against
chom_mlp_loss_grad (the handle's allocated buffers), through the C ABI.

Both run the same kernels on the same device inputs, so the gradient must agree
to the last bit up to the order of the loss's workgroup sum; two calls in a row,
the second with fewer records (the static workspace keeps the first call's
contents, which must not leak into the second), and a size above the workspace
limit must be refused before any device work.
"""
import numpy as np
import pytest

import chom_inputs as ci
from gpu_util import banner, require_gpu
from mlp_util import norm_record, rows, weights
from oracle import mlp as ref

pytestmark = pytest.mark.gpu


def _targets(n, seed):
    u = rows(seed, n, 33, stream=1)
    y_mu = np.concatenate([np.linspace(1.0, 8.0, 21), np.linspace(0.2, 0.6, 6), np.linspace(0.3, 0.9, 6)])
    y = y_mu + 0.2 * y_mu * u
    return y[:, :21].copy(), y[:, 21:27].copy(), y[:, 27:].copy()


def test_noalloc_gradient_equals_allocating_entry_point():
    torch = require_gpu()
    from paper_1610_03484_amd import Surrogate
    from paper_1610_03484_amd import _lib as L
    n_max = 3000
    params = ci.draw_params(23, n_max)
    C, K, D = _targets(n_max, 24)
    x_mu, x_sd = ref.column_stats(ref.features(params))
    y_mu, y_sd = ref.column_stats(ref.encode(ref.targets(C, K, D)))
    s = Surrogate(members=2, seed=0, device=True)
    s.set_weights(0, weights(41))
    s.set_weights(1, weights(40))
    s.set_normalisation(norm_record(x_mu, x_sd, y_mu, y_sd))
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    nparam = s.sizes()[0]
    for n, member in ((n_max, 1), (700, 0)):
        banner(f"no-alloc loss/gradient vs allocating entry point: n={n}, member={member}")
        p, c, k, d = dev(params[:n]), dev(C[:n]), dev(K[:n]), dev(D[:n])
        loss_a, g_a = s.loss_grad(member, p, c, k, d)
        loss_t = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        grad_t = torch.full((nparam,), float("nan"), dtype=torch.float32, device="cuda")
        s.loss_grad_noalloc(member, p, c, k, d, loss_t, grad_t)
        torch.cuda.synchronize()
        loss_b, g_b = float(loss_t.cpu()[0]), grad_t.cpu().numpy()
        same = int(np.sum(g_a == g_b))
        banner(f"  loss {loss_a:.10e} vs {loss_b:.10e}; gradient entries equal {same}/{nparam}, "
               f"max |diff| {np.abs(g_a - g_b).max():.2e}")
        assert np.all(np.isfinite(g_b))
        assert abs(loss_a - loss_b) <= 1e-12 * abs(loss_a)
        assert np.abs(g_a - g_b).max() <= 1e-6 * np.abs(g_a).max()
    banner("no-alloc: a call above the workspace limit is refused")
    big = dev(np.repeat(params[:1], 4097, axis=0))
    with pytest.raises(L.ChomError) as ei:
        s.loss_grad_noalloc(0, big, dev(np.repeat(C[:1], 4097, axis=0)), dev(np.repeat(K[:1], 4097, axis=0)),
                            dev(np.repeat(D[:1], 4097, axis=0)), loss_t, grad_t)
    assert ei.value.status == L.CHOM_EINVAL
    s.close()
