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
        print(f"[gpu] shapes level={level} flux={flux} variant={v} rows={dk.Context.shape_rows(n, v)}", flush=True)
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
