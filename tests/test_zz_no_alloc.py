"""fetd_batch_step_noalloc (the entry point for callers that cannot
allocate) against fetd_batch_step on the same runs: deterministic mode, so
bit for bit; two calls in a row, the second with fewer and smaller runs;
nothing allocated (torch's allocator, which the library's simulations draw
from, holds the same bytes before and after each call)."""
import numpy as np
import pytest

from paper_1707_04333_amd import inputs as I

pytestmark = pytest.mark.gpu


def _state(g):
    out = {name: g.field(name) for name in ("e", "d", "b", "j")}
    for si in range(2):
        p = g.particles(si)
        for k in ("id", "tri", "slot", "lam", "u"):
            out[f"{k}{si}"] = p[k]
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_batch_step(precision):
    import torch
    from paper_1707_04333_amd import fetdpic as fp
    calls = [([(12, 0.02, 3001, 0.3), (20, 0.03, 9000, 0.1), (9, 0.015, 1500, 1.0)], 17),
             ([(8, 0.012, 700, 0.5), (10, 0.016, 1201, 0.2)], 9)]
    for specs, steps in calls:
        wls = [I.pair_plasma(n_side=n, length=L, n_pairs=p, theta=t, steps=steps,
                             precision=precision) for n, L, p, t in specs]
        ref = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=4)
               for w in wls]
        got = [fp.from_workload(w, spai_level=1, deterministic=True, resort_every=4)
               for w in wls]
        for g in ref + got:
            g.diagnostics()
        b = fp.Batch(ref, use_graph=False)
        b.step(steps, "vay")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        fp.batch_step_noalloc(got, steps, "vay")
        got[0].sync()
        assert torch.cuda.memory_allocated() == before
        for gr, gg in zip(ref, got):
            a, c = _state(gr), _state(gg)
            for k in a:
                assert np.array_equal(a[k], c[k]), k
            assert gg.diagnostics()["gauss_rel"] <= (1e-12 if precision == "fp64" else 1e-6)
        b.close()
        for g in ref + got:
            g.close()
