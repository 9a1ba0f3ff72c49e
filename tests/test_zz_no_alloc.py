"""The allocation-free proposal forward (activations in the library's static
device array) against prrtc_proposal_forward, through the C ABI: two calls in
a row, the second smaller (matrix-core GEMM path, then the small-batch path),
and the size limit."""
import sys

import numpy as np
import pytest

from paper_2503_06757_amd import proposal as PR
from paper_2503_06757_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(torch, rng, robot, n_scenes, n):
    dof = W.robot_dof(robot)
    scene_of = rng.integers(0, n_scenes, n).astype(np.int32)
    s = rng.uniform(robot["q_lo"], robot["q_hi"], (n, dof)).astype(np.float32)
    g = rng.uniform(robot["q_lo"], robot["q_hi"], (n, dof)).astype(np.float32)
    return {k: torch.from_numpy(v).cuda() for k, v in dict(scene_of=scene_of, s=s, g=g).items()}


def _run(P, ctx, torch, fn, mid, rid, vox_t, n_scenes, t, n, cw):
    out = torch.full((n, cw), float("nan"), dtype=torch.float32, device="cuda")
    fn(ctx, mid, rid, vox_t.data_ptr(), n_scenes, t["scene_of"].data_ptr(), t["s"].data_ptr(),
       t["g"].data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_forward_equals_forward(gpu, r7, r14):
    P, ctx, torch = gpu
    rng = np.random.default_rng(41)
    for robot, seed in ((r7, 3), (r14, 4)):
        dof = W.robot_dof(robot)
        cw = 8 * (1 + 2 * dof)
        params = PR.init_params(dof, seed)
        for k in ("bv", "b1", "b2", "b3", "b4"):
            params[k] = (rng.standard_normal(params[k].shape) * 0.1).astype(np.float32)
        mid = P.prrtc_load_proposal(ctx, PR.pack(params, dof))
        rid = P.prrtc_load_robot(ctx, robot)
        scenes = [W.scene_mixed(0x5A000000 + i, robot, 8 + 16 * i) for i in range(7)]
        vox_t = torch.zeros((len(scenes), 4096), dtype=torch.uint8, device="cuda")
        for i, prims in enumerate(scenes):
            sid = P.prrtc_load_scene(ctx, prims)
            P.prrtc_voxelize(ctx, sid, vox_t[i].data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        # 200 samples over 7 scenes (GEMMs, ragged against 64-row tiles), then 5 over 2 (one workgroup per row)
        for n_scenes, n in ((7, 200), (2, 5)):
            say("noalloc forward: dof %d, %d samples over %d scenes" % (dof, n, n_scenes))
            t = _inputs(torch, rng, robot, n_scenes, n)
            want = _run(P, ctx, torch, P.prrtc_proposal_forward, mid, rid, vox_t, n_scenes, t, n, cw)
            got = _run(P, ctx, torch, P.prrtc_proposal_forward_noalloc, mid, rid, vox_t, n_scenes, t, n, cw)
            assert np.all(np.isfinite(want))
            assert np.array_equal(got, want)      # the same kernels on the same inputs
        # beyond the static array's limits: refused before any work
        for n_scenes, n in ((1, 257), (257, 4)):
            t = _inputs(torch, rng, robot, 1, n)
            with pytest.raises(P.PrrtcError) as e:
                _run(P, ctx, torch, P.prrtc_proposal_forward_noalloc, mid, rid, vox_t, n_scenes, t, n, cw)
            assert e.value.status == P.PRRTC_E_ARG
            assert "static scratch" in P.prrtc_last_error(ctx)
