"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle on the same seeded scene."""
import numpy as np
import pytest

# parity bar (forward): features of unit-variance inputs and alpha
TOL_FEAT = 2e-4
TOL_ALPHA = 1e-5


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_render(scene, rast=None, bg=None, lists=True):
    """Render `scene` on cuda:0; returns numpy arrays and the rasterizer."""
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    print(f"[gpu] render {scene.name} n={scene.n} c={scene.c} "
          f"{scene.cam.width}x{scene.cam.height}", flush=True)
    g = GaussianSoA.from_scene(scene)
    if rast is None:
        rast = Rasterizer(0, max_n=max(1, scene.n), max_w=scene.cam.width, max_h=scene.cam.height)
    bgt = None if bg is None else torch.as_tensor(bg, dtype=torch.float32, device="cuda")
    feat, alpha = rast.forward(g, scene.cam, bgt)
    T, last = rast.pixel_state(scene.cam)
    out = dict(feat=feat.cpu().numpy(), alpha=alpha.cpu().numpy(), T=T.cpu().numpy(),
               last=last.cpu().numpy(), n_keys=rast.n_keys)
    if lists:
        ts, so = rast.tile_lists(scene.cam)
        out["tile_start"] = ts.cpu().numpy().astype(np.int64)
        out["sorted"] = so.cpu().numpy()
    torch.cuda.synchronize()
    return out, rast, g


def compare_lists(gpu, ora):
    start, lst = ora.tile_lists()
    np.testing.assert_array_equal(gpu["tile_start"], start)
    np.testing.assert_array_equal(gpu["sorted"], lst)


def compare_forward(gpu, ora, ref=None, bg=None, tol_feat=TOL_FEAT, tol_alpha=TOL_ALPHA,
                    check_last=True):
    """Element-wise forward parity.  Pixels with a near-threshold decision
    (flagged by the oracle) must match one of the oracle's branch variants.
    Returns a small report dict."""
    ref = ora.render(bg=bg) if ref is None else ref
    F, A = gpu["feat"].astype(np.float64), gpu["alpha"].astype(np.float64)
    dF = np.abs(F - ref["feat"]).max(0)
    dA = np.abs(A - ref["alpha"])
    flagged = ref["nflags"] > 0
    ok = (dF <= tol_feat) & (dA <= tol_alpha)
    bad = ~ok & ~flagged
    assert not bad.any(), (
        f"{bad.sum()} unflagged pixels off: max dF {dF[~flagged].max():.3g} "
        f"max dA {dA[~flagged].max():.3g} at {np.argwhere(bad)[:5].tolist()}")
    # last contributor is an index: exact where no decision was near a threshold
    if check_last:
        np.testing.assert_array_equal(gpu["last"][~flagged], ref["last"][~flagged])
    excluded = 0
    for (y, x) in np.argwhere(flagged & ~ok):
        var = ora.pixel_variants(int(x), int(y), bg=bg)
        if var is None:
            excluded += 1
            continue
        want = np.concatenate([F[:, y, x], [A[y, x]]])
        d = np.abs(var - want[None])
        hit = (d[:, :-1].max(1) <= tol_feat) & (d[:, -1] <= tol_alpha)
        assert hit.any(), f"flagged pixel {(x, y)} matches no branch variant: {d.max(1)}"
    assert excluded <= max(2, flagged.size // 100000), excluded
    return dict(max_dF=float(dF[~flagged].max()) if (~flagged).any() else 0.0,
                max_dA=float(dA[~flagged].max()) if (~flagged).any() else 0.0,
                flagged=int(flagged.sum()), excluded=excluded)
