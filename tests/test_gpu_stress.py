"""GPU parity of the stress workload over four consecutive frames: the
realistic generator at 2048^2 per view (about 7.55M Gaussians, 17.8M keys,
C = 32, 2048^2 target), the features of frame k perturbed by N(0, 0.05) and
the geometry unchanged.  The four frames go through the serving loop as one
batch, forward and adjoint, frames 1-3 reusing frame 0's projection and
sorted lists (their geometry is byte-identical).  Everything is compared
with the plain path and with the oracle."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import compare_backward, compare_forward, compare_grads, torch_cuda

pytestmark = pytest.mark.gpu

FRAMES = 4


def test_stress_four_frames_served_forward_and_backward():
    """The four frames of one stream, each with its own dL/dF ~ N(0, 1),
    submitted back to back with sharing allowed, are served as one batch
    with the adjoint; frames 1-3 share frame 0's sort.  Each served image
    equals its plain render bit for bit and matches the oracle (features,
    alpha, last contributor); each served gradient matches the plain
    adjoint within the gradient bar and the oracle's FP64 gradients of every
    Gaussian (the oracle differentiating the branch the GPU took at
    near-threshold decisions)."""
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer, empty_grads
    from paper_2405_14866_amd.serve import Server
    base = scenes.make_cfg5()
    frames = [scenes.make_cfg5(frame=k, base=base) for k in range(FRAMES)]
    n, c, W, H = base.n, base.c, base.cam.width, base.cam.height
    print(f"[gpu] stress serve fwd+bwd {FRAMES} x n={n} {W}x{H}", flush=True)
    gs = [GaussianSoA.from_scene(sc) for sc in frames]
    outs = [(torch.empty((c, H, W), device="cuda"), torch.empty((H, W), device="cuda"))
            for _ in frames]
    ups = [scenes.make_cfg3_upstream(60 + k, c, H, W) for k in range(FRAMES)]
    dFs = [torch.as_tensor(u, device="cuda") for u in ups]
    grads = [empty_grads(n, c) for _ in frames]
    srv = Server(0, c=c, slots=1, max_batch=FRAMES, max_gauss_per_batch=FRAMES * n + 8192,
                 max_keys_per_batch=int(2.6 * FRAMES * n), max_pixels_per_batch=FRAMES * W * H,
                 max_side=max(W, H), keys_per_gaussian=2.5, batch_window_us=300000, backward=True)
    torch.cuda.synchronize()
    tickets = [srv.submit(g, sc.cam, f, a, stream_id=0, d_feat=dF, grads=gr, share=True)
               for sc, g, (f, a), dF, gr in zip(frames, gs, outs, dFs, grads)]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    assert all(r.status == 0 for r in results), [r.status for r in results]
    print("batch sizes", [r.batch_size for r in results], "shared", [r.shared for r in results], flush=True)
    assert all(r.batch_size == FRAMES for r in results)
    assert [r.shared for r in results] == [False] + [True] * (FRAMES - 1)

    rast = Rasterizer(0, max_n=n, max_w=W, max_h=H, keys_per_gaussian=2.5)
    for k, (sc, g, (fs, as_)) in enumerate(zip(frames, gs, outs)):
        print(f"[gpu] stress frame {k}: plain forward + backward", flush=True)
        feat, alpha = rast.forward(g, sc.cam)
        assert torch.equal(feat, fs) and torch.equal(alpha, as_), k
        T, last = rast.pixel_state(sc.cam)
        plain = rast.backward(g, dFs[k])
        torch.cuda.synchronize()
        got = {key: v.cpu().numpy() for key, v in grads[k].items()}
        compare_grads(got, {key: v.cpu().numpy() for key, v in plain.items()}, np.zeros(0, np.int64))
        gpu = dict(feat=feat.cpu().numpy(), alpha=alpha.cpu().numpy(), T=T.cpu().numpy(),
                   last=last.cpu().numpy())
        ora = oracle.Oracle(sc)
        ref_fwd = ora.render()
        rep = compare_forward(gpu, ora, ref=ref_fwd)
        worst, undet, loose = compare_backward(got, gpu, ora, ups[k], ref_fwd=ref_fwd)
        print(f"frame {k}", rep, "served grads vs oracle, worst", worst, "undetermined pixels", undet,
              "loose Gaussians", loose, flush=True)
        ora.close()
