"""The allocation-free entry point (dk_mlmc_level_pair_noalloc) against dk_mlmc_level_pair: identical
per-sample values and moment sums equal to rounding, on two calls in a row (the second smaller),
through the C ABI, for single paths and pairs, FP32 and FP64 states, and 29 observables."""
import numpy as np
import pytest

import dk_workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_08872_amd as dk  # noqa: E402


def moments_array(ms):
    return np.array([[m.count] + list(m.sums) for m in ms])


@pytest.mark.parametrize("name,problem,calls", [
    # (level, first, count): the finest config-2 pair, then a smaller batch of a shallower pair
    ("config2", W.config2(N=1e4).with_(seed=3), [(4, 5, 300), (2, 0, 97)]),
    # single paths on level 0 (many per launch), then a smaller batch
    ("config2-l0", W.config2(N=1e4).with_(seed=4), [(0, 11, 70000), (0, 3, 1000)]),
    # 29 observables (config 3, uncentred, a squared bump), 64^2 pairs then 32^2 pairs
    ("config3", W.config3(N=1e3).with_(levels=5, seed=5), [(3, 0, 200), (2, 7, 50)]),
    # FP64 state, the paper's setting (2 pi torus, centred sqrt(N)-scaled observable)
    ("paper-f64", W.paper_reg(2e9).with_(seed=6), [(5, 0, 24), (3, 1, 10)]),
])
def test_noalloc_matches_level_pair(name, problem, calls):
    ctx = dk.Context(0)
    for level, first, count in calls:
        print(f"[gpu] {name}: level {level}, samples [{first}, +{count})", flush=True)
        sa, pa = dk.level_pair_noalloc(problem, level, first, count, per_sample=True)
        sb, pb = dk.level_pair(problem, level, first, count, per_sample=True, ctx=ctx)
        torch.cuda.synchronize()
        assert torch.equal(pa, pb), f"{name} level {level}: per-sample values differ"
        ma, mb = moments_array(sa), moments_array(sb)
        assert np.array_equal(ma[:, 0], mb[:, 0])
        scale = np.maximum(np.abs(ma[:, 1:]), np.abs(mb[:, 1:])) + 1e-300
        assert np.all(np.abs(ma[:, 1:] - mb[:, 1:]) <= 1e-12 * scale), f"{name} level {level}: moment sums differ"
        # without a per-sample output (the values go to the library's fixed workspace)
        sc = dk.level_pair_noalloc(problem, level, first, count)
        torch.cuda.synchronize()
        mc = moments_array(sc)
        assert np.all(np.abs(mc[:, 1:] - mb[:, 1:]) <= 1e-12 * scale), f"{name} level {level}: moment sums differ"
    ctx.close()


def test_noalloc_refuses_what_it_does_not_run():
    p = W.config3(N=1e5)          # level 5 is 256 x 256, a streamed grid
    with pytest.raises(dk.DKError):
        dk.level_pair_noalloc(p, 5, 0, 4)
    with pytest.raises(dk.DKError):
        dk.level_pair_noalloc(W.config2(), 5, 0, 4)      # no level 5
