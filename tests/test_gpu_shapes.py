"""Every tile-shape variant of the resident kernel computes the same sample paths.

This doubles as a race detector: the variants split each sample over different numbers of
lanes, wavefronts and LDS halo rows, so a missing barrier or a wrong halo index shows up as a
difference.  Fields must be bit-identical; observables differ only through the order of the
FP64 lane reduction.
"""
import numpy as np
import pytest

import dk_workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2311_08872_amd as dk  # noqa: E402


@pytest.mark.parametrize("flux", [W.FLUX_CENTRAL, W.FLUX_STAGGERED])
@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_shape_variants_agree(level, flux):
    p = W.config2(N=2e3).with_(T=0.05 / 16 if level >= 3 else 0.05, flux=flux)   # shorter horizon on big levels
    ctx = dk.Context(0)
    n = p.n(level)
    coupled = level >= 1
    count = 37 if n >= 64 else 301                          # ragged against every block size
    ref = None
    v = 0
    while dk.Context.shape_rows(n, v) > 0:
        print(f"[gpu] shapes level={level} flux={flux} variant={v} rows={dk.Context.shape_rows(n, v)} "
              f"spw={dk.Context.shape_spw(n, v)}", flush=True)
        ctx.set_shape(n, v)
        out = dk.level_fields(p, level, coupled, 11, count, ctx=ctx)
        torch.cuda.synchronize()
        out = [o.cpu().numpy() if o is not None else None for o in out]
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[1].view(np.uint32), ref[1].view(np.uint32)), v
            if coupled:
                assert np.array_equal(out[2].view(np.uint32), ref[2].view(np.uint32)), v
            assert np.allclose(out[0], ref[0], rtol=1e-11, atol=1e-14), v
        v += 1
    assert v >= 2
    ctx.close()


def test_tuning_choices_round_trip_through_json(tmp_path, monkeypatch, capfd):
    """The autotuner's choice is exported as JSON, a fresh context that loads the text uses it
    without timing, the DK_TUNE_CACHE file is written and read, and bad text is rejected."""
    import json
    monkeypatch.setenv("DK_LOG", "1")
    cache = tmp_path / "shapes.json"
    monkeypatch.setenv("DK_TUNE_CACHE", str(cache))
    p = W.config2(N=1e4)
    ctx = dk.Context(0)
    dk.level_pair(p, 4, 0, 720, ctx=ctx)          # 1.03e11 cell updates: large enough to be tuned
    assert "tuned n=128" in capfd.readouterr().err
    text = ctx.tuning_json()
    j = json.loads(text)
    entry = [e for e in j["shapes"] if e["n"] == 128 and e["pair"] == 1 and e["flux"] == p.flux]
    assert j["format"] == "dk-tile-shapes-1" and j["arch"].startswith("gfx") and len(entry) == 1
    rows = entry[0]["rows"]
    assert rows in (8, 16)
    ctx.close()
    assert json.loads(cache.read_text()) == j      # DK_TUNE_CACHE rewritten after the choice

    ctx2 = dk.Context(0)                           # loads DK_TUNE_CACHE when created
    assert json.loads(ctx2.tuning_json()) == j
    dk.level_pair(p, 4, 0, 720, ctx=ctx2)
    assert "tuned n=128" not in capfd.readouterr().err
    st = [s for s in ctx2.stats() if s["level"] == 4]
    assert st and st[0]["rows"] == rows
    with pytest.raises(dk.DKError):
        ctx2.load_tuning_json(text.replace(j["arch"], "gfx000"))
    with pytest.raises(dk.DKError):
        ctx2.load_tuning_json(text.replace(f'"rows": {rows}', '"rows": 3'))
    with pytest.raises(dk.DKError):
        ctx2.load_tuning_json("{}")
    ctx2.close()

    monkeypatch.delenv("DK_TUNE_CACHE")
    ctx3 = dk.Context(0)
    assert json.loads(ctx3.tuning_json())["shapes"] == []
    ctx3.load_tuning_json(text)
    assert json.loads(ctx3.tuning_json()) == j
    ctx3.close()


def test_tuning_json_samples_per_block_entries():
    """A shape entry may name its samples per block: an existing (rows, spw) pair selects that
    variant, one that no compiled shape has is rejected, and an entry without spw names the
    ~256-lane shape with that row count."""
    import json
    n = 64
    wide = [v for v in range(4) if dk.Context.shape_rows(n, v) == 8 and dk.Context.shape_spw(n, v) == 4]
    assert wide, "the 64^2 kernel has a 1024-lane 8-row shape"
    assert dk.Context.shape_spw(n, 0) == 1 and dk.Context.shape_rows(n, 0) == 8

    def doc(entry):
        return json.dumps({"format": "dk-tile-shapes-1", "arch": arch, "shapes": [entry]})

    ctx = dk.Context(0)
    arch = json.loads(ctx.tuning_json())["arch"]
    ctx.load_tuning_json(doc({"n": n, "pair": 1, "flux": 0, "rows": 8, "spw": 4}))
    got = json.loads(ctx.tuning_json())["shapes"]
    assert {"n": n, "pair": 1, "flux": 0, "rows": 8, "spw": 4} in got
    ctx.load_tuning_json(doc({"n": n, "pair": 1, "flux": 0, "rows": 8}))
    got = json.loads(ctx.tuning_json())["shapes"]
    assert {"n": n, "pair": 1, "flux": 0, "rows": 8, "spw": 1} in got
    with pytest.raises(dk.DKError):
        ctx.load_tuning_json(doc({"n": n, "pair": 1, "flux": 0, "rows": 8, "spw": 3}))
    ctx.close()
