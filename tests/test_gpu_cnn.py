"""GPU checks of the control-variate network kernels (BF16 MFMA, FP32 accumulation) against
the FP64 reference network, and of the control-variate estimator's unbiasedness.

Tolerances.  The two 16->16 convolutions take BF16 operands (8 significant bits: each rounding
is at most 2^-9 = 2e-3 relative) and accumulate in FP32; the first convolution, pooling and MLP
run in FP32.  One rounding of each operand and of each layer's output gives at most
3 x 2^-9 = 5.9e-3 relative per 16->16 layer on every product, and the two layers' errors add
in the output; the sums over 144 products cancel only partly for these random weights and inputs
(both layers' terms have one sign after the ReLU in about half of them), so the forward output is
held to 1e-2 of its RMS (the bar of the scope's CNN parity item; measured 2.2e-3 .. 3.7e-3).  The
backward pass runs the same BF16 products twice more (input gradients and weight gradients), so
each gradient block is held to 3e-2 of its norm (measured 4.5e-3 .. 1.5e-2) and the loss to 1e-2.
"""
import math

import numpy as np
import pytest

import dk_workloads as W
from oracle import cnn as ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_08872_amd as dk  # noqa: E402


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


def rand_params(seed):
    p = dk.cnn_init(seed)
    rng = np.random.default_rng(seed + 100)
    # non-zero biases so that every parameter block carries gradient
    for off, cnt in [(144, 16), (2464, 16), (4784, 16), (5824, 64), (5952, 1)]:
        p[off:off + cnt] = 0.1 * rng.standard_normal(cnt)
    return p


@pytest.mark.parametrize("n,batch", [(16, 64), (32, 24), (8, 300)])
def test_forward_matches_fp64_reference(n, batch):
    banner(f"cnn forward n={n} batch={batch}")
    p = rand_params(n)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((batch, n, n)).astype(np.float32)
    r = dk.cnn_forward(p, torch.from_numpy(x).cuda()).cpu().numpy()
    rr = ref.forward(ref.unflatten(p.astype(np.float64)), x.astype(np.float64))
    rms = np.sqrt(np.mean(rr ** 2))
    banner(f"forward max error / RMS = {np.max(np.abs(r - rr)) / rms:.3g}")
    assert np.max(np.abs(r - rr)) <= 1e-2 * rms, (np.max(np.abs(r - rr)), rms)


@pytest.mark.parametrize("n,batch", [(16, 48), (32, 16)])
def test_gradient_matches_fp64_reference(n, batch):
    banner(f"cnn gradient n={n} batch={batch}")
    p = rand_params(7 + n)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((batch, n, n)).astype(np.float32)
    y = rng.standard_normal(batch).astype(np.float32)
    loss, g = dk.cnn_loss_grad(p, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    lr_, gr = ref.loss_and_grad(ref.unflatten(p.astype(np.float64)), x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lr_) <= 1e-2 * lr_
    gd = ref.unflatten(g.astype(np.float64))
    worst = 0.0
    for k in ref.ORDER:
        num = np.linalg.norm(gd[k] - gr[k])
        den = np.linalg.norm(gr[k])
        worst = max(worst, num / max(den, 1e-30))
        assert num <= 3e-2 * den + 1e-7, (k, num / max(den, 1e-30))
    banner(f"loss relative error {abs(loss - lr_) / lr_:.3g}; largest gradient-block relative error {worst:.3g}")


def test_training_reduces_loss_and_keeps_estimator_unbiased():
    """Training on the level-2 pairs of config 2 lowers the training loss; with the trained and
    with an untrained network the control-variate MLMC estimate agrees with plain MLMC
    (the control variate is unbiased for any fixed network)."""
    p = W.config2(N=1e4).with_(levels=3)
    banner("cv_train level 2 (4096 pairs)")
    res = dk.cv_train(p, 2, n_train=4096, epochs=6, batch=128, lr=2e-3, n_val=2048, seed=0)
    assert res["loss"][-1] < res["loss"][0]
    assert res["var_Y_minus_r"] < 1.05 * res["var_Y"]
    params = np.zeros((p.levels, dk.L.DK_CNN_NPARAM), np.float32)
    params[2] = res["params"]
    params[1] = rand_params(3)                       # an untrained network on level 1
    banner("estimates: plain and control variate")
    plain = dk.estimate(p, 6e-3, L_start=2)
    cv = dk.estimate(p, 6e-3, L_start=2, cv_params=params, cv_level_mask=0b110, cv_ratio=4)
    assert plain["L"] == 2 and cv["L"] == 2
    se = math.sqrt(plain["var_est"][0] + cv["var_est"][0])
    assert abs(plain["estimate"][0] - cv["estimate"][0]) < 4.5 * se
    # level by level
    for l in (1, 2):
        se_l = math.sqrt(plain["Vhat"][l] / plain["M"][l] + cv["Vhat"][l] / cv["M"][l])
        assert abs(plain["Yhat"][l] - cv["Yhat"][l]) < 4.5 * se_l, l


def test_control_variate_gain_is_measured():
    """What the trained network buys on config 2 (pair 1, coarse 8x8 input): the fraction of
    Var(Y_1) it removes on held-out pairs is reported; it cannot be negative beyond noise and
    the estimator's variance Var(Y - r) + Var(r)/k is compared with Var(Y)."""
    p = W.config2(N=1e4)
    res = dk.cv_train(p, 1, n_train=1 << 14, epochs=6, batch=256, lr=1e-3, n_val=1 << 13, seed=1)
    vy, vd, vr = res["var_Y"], res["var_Y_minus_r"], res["var_r"]
    print(f"[gpu] cv gain level 1: Var(Y)={vy:.4g} Var(Y-r)={vd:.4g} Var(r)={vr:.4g} "
          f"explained={(1 - vd / vy):.3%}", flush=True)
    se = vy * math.sqrt(2.0 / (1 << 13))
    assert vd <= vy + 4.5 * se
    assert vd + vr / 4 <= 1.1 * vy
