"""trace_rays_noalloc (the entry point that allocates nothing) against trace_rays.

Both run the same kernels, and every ray's result depends only on that ray, so
the outputs must be bitwise equal.  Two calls in a row share the GPU's static
scratch: the second, smaller one must not see the first's counters, queues or
status.  The oracle bar is covered by trace_rays' own parity tests; here one
sampled set of rows is also checked against the oracle directly.
"""

import numpy as np
import pytest

import nnm_inputs as ni
import paper_2201_09147_amd as nnm
from oracle import tracing as orc
from tests.parity import check_fp32, check_lowp, compare

pytestmark = pytest.mark.gpu


def _outputs(n, m, dev):
    import torch
    return {
        "depth": torch.full((n,), -1.0, dtype=torch.float32, device=dev),
        "hit": torch.full((n,), 7, dtype=torch.uint8, device=dev),
        "normal": torch.full((n, 3), -2.0, dtype=torch.float32, device=dev),
        "steps": torch.full((n, m), 255, dtype=torch.uint8, device=dev),
        "status": torch.full((n,), 255, dtype=torch.uint8, device=dev),
    }


def _run(entry, stack, params, o, v, with_status=True):
    import torch
    dev = torch.device("cuda", 0)
    out = _outputs(o.shape[0], stack.m, dev)
    entry(stack, params, o, v, None, out["depth"], out["hit"], out["normal"], out["steps"],
          out["status"] if with_status else None)
    torch.cuda.synchronize()
    res = {k: t.cpu().numpy() for k, t in out.items()}
    if not with_status:
        res.pop("status")
    return res


def _bitwise_equal(a, b, tag):
    for k in a:
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, (tag, k)
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), (tag, k)


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_noalloc_matches_trace_rays_two_calls(precision):
    import torch
    dev = torch.device("cuda", 0)
    big = ni.make_scene("stack3_1080p")          # 2,073,600 rays: the largest the scratch holds is 2^21
    small = ni.make_scene("stack3_512sq").with_size(300, 173)  # ragged tail: 51,900 rays
    stack = nnm.load_siren_stack(big, precision, 0)
    p = nnm.TraceParams(big.step_scale, big.eps, big.far, big.max_steps)
    try:
        calls = []
        for k, (scene, with_status) in enumerate(((big, True), (small, False))):
            o, v, _ = scene.rays()
            assert o.shape[0] <= nnm.NOALLOC_MAX_RAYS
            og, vg = torch.from_numpy(o).to(dev), torch.from_numpy(v).to(dev)
            print(f"call {k}: {precision} {o.shape[0]} rays, status {'given' if with_status else 'in scratch'}",
                  flush=True)
            ref = _run(nnm.trace_rays, stack, p, og, vg, with_status)
            got = _run(nnm.trace_rays_noalloc, stack, p, og, vg, with_status)
            _bitwise_equal(got, ref, f"call {k}")
            assert got["hit"].sum() > 0.1 * o.shape[0]
            calls.append((scene, o, v, got))
        # the second (smaller) call against the oracle on a row sample
        scene, o, v, got = calls[1]
        rows = np.arange(1, 173, 9)
        idx = (rows[:, None] * 300 + np.arange(300)[None, :]).ravel()
        r = orc.trace(scene, o[idx], v[idx])
        st = compare({k: a[idx] for k, a in got.items()}, r)
        print(f"noalloc {precision} vs oracle: {st}")
        (check_fp32 if precision == "fp32" else check_lowp)(st)
    finally:
        stack.close()


def test_noalloc_rejects_oversize_and_profiler():
    import torch
    dev = torch.device("cuda", 0)
    scene = ni.make_scene("stack3_512sq")
    stack = nnm.load_siren_stack(scene, "bf16", 0)
    try:
        n = nnm.NOALLOC_MAX_RAYS + 1
        o = torch.zeros((n, 3), dtype=torch.float32, device=dev)
        v = torch.zeros((n, 3), dtype=torch.float32, device=dev)
        out = _outputs(n, stack.m, dev)
        with pytest.raises(nnm.NnmError, match="static scratch"):
            nnm.trace_rays_noalloc(stack, nnm.TraceParams(), o, v, None, out["depth"], out["hit"])
        prof = nnm.Profiler()
        with pytest.raises(nnm.NnmError, match="profiler"):
            nnm.trace_rays_noalloc(stack, nnm.TraceParams(profiler=prof), o[:8], v[:8], None, out["depth"][:8],
                                   out["hit"][:8])
        prof.close()
        # nothing was launched: the outputs keep their fill values
        torch.cuda.synchronize()
        assert float(out["depth"][:8].min()) == -1.0
    finally:
        stack.close()
