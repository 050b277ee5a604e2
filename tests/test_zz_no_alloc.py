"""The no-allocation frame (vplmc_render_static) against vplmc_render with a
caller workspace: two calls in a row on the library's static workspace, the
second with fewer slices, each bit-identical to the same frame rendered on a
workspace tensor (the same kernels; the completion's sums are order-fixed)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from _gpu_common import log  # noqa: E402
from paper_2202_12567_amd import api  # noqa: E402
from paper_2202_12567_amd import _native as N  # noqa: E402
from scenegen import make_scene, scene_sample  # noqa: E402


def test_static_workspace_frame_equals_the_caller_workspace_frame():
    dev = torch.device("cuda", 0)
    full = make_scene("tiny", 4)
    ctx = api.Context(0)
    ctx.set_occluders(full.spheres)
    prm = api.default_params(seed=4, max_iter=30, fixed_iters=True)
    cases = [("16 slices", full), ("4 slices", scene_sample(full, [1, 6, 11, 12]))]
    for name, sc in cases:
        plan = api.Plan(sc, prm)
        assert plan.workspace_bytes <= (64 << 20)
        ds = api.DeviceScene(sc, dev)
        log(f"static workspace frame: {name}, workspace {plan.workspace_bytes / 2**20:.1f} MiB")
        ws = api.workspace(plan, dev)
        ref = api.render(ctx, plan, ds, prm, ws).clone()
        got = torch.full((sc.m, 3), -1.0, dtype=torch.float32, device=dev)
        api.render_static(ctx, plan, ds, prm, got)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), f"{name}: max diff {(got - ref).abs().max().item():.3e}"
        assert float(ref.abs().sum()) > 0.0


def test_static_workspace_rejects_a_frame_above_its_size():
    dev = torch.device("cuda", 0)
    sc = make_scene("tiny", 4)
    ctx = api.Context(0)
    prm = api.default_params(seed=4, pass1_ppm=500000, pass2_ppm=500000)
    plan = api.Plan(sc, prm)
    assert plan.workspace_bytes > (64 << 20)
    ds = api.DeviceScene(sc, dev)
    with pytest.raises(N.VplmcError) as e:
        api.render_static(ctx, plan, ds, prm)
    assert e.value.code == N.EINVAL and "static workspace" in str(e.value)
