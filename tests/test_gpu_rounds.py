"""Algorithm 1 with each round's levels run concurrently (one stream per level) or captured into
a hipGraph launched once per round gives exactly the results of the level-by-level run: the
samples, their chunking and the ordered sums are the same."""
import pytest

import dk_workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_08872_amd as dk  # noqa: E402


@pytest.mark.parametrize("name,problem,eps", [
    ("config2", W.config2(N=1e4).with_(seed=7), 1e-2),
    ("config3", W.config3(N=1e5).with_(levels=5, seed=3), 2e-3),
])
def test_round_modes_identical(name, problem, eps):
    res = []
    for mode in (0, 1, 2):
        print(f"[gpu] {name} round_mode={mode}", flush=True)
        ctx = dk.Context(0)
        r = dk.estimate(problem, eps, ctx=ctx, round_mode=mode)
        ctx.close()
        res.append(r)
    for r in res[1:]:
        assert r["M"] == res[0]["M"]
        assert r["L"] == res[0]["L"]
        assert r["estimate"] == res[0]["estimate"]
        assert r["Yhat"] == res[0]["Yhat"] and r["Vhat"] == res[0]["Vhat"]
    assert len(res[0]["estimate"]) == len(problem.obs)
