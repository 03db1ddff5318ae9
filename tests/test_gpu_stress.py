"""GPU parity of the stress workload over four consecutive frames: the
realistic generator at 2048^2 per view (about 7.55M Gaussians, 17.8M keys,
C = 32, 2048^2 target), the features of frame k perturbed by N(0, 0.05).
The four forwards go through the serving loop as one batch; each frame's
adjoint runs on a plain frame.  Everything is compared with the oracle."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import compare_backward, compare_forward, torch_cuda

pytestmark = pytest.mark.gpu

FRAMES = 4


def test_stress_four_frames_served_and_differentiated():
    """The four frames submitted back to back from four streams are served in
    batches (all four fit one slot); each served image equals its plain
    render bit for bit and matches the oracle (features, alpha, last
    contributor).  Each frame's adjoint under its own dL/dF ~ N(0, 1) matches
    the oracle's FP64 gradients of every Gaussian (the oracle differentiating
    the branch the GPU took at near-threshold decisions)."""
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    from paper_2405_14866_amd.serve import Server
    base = scenes.make_cfg5()
    frames = [scenes.make_cfg5(frame=k, base=base) for k in range(FRAMES)]
    n, c, W, H = base.n, base.c, base.cam.width, base.cam.height
    print(f"[gpu] stress serve {FRAMES} x n={n} {W}x{H}", flush=True)
    gs = [GaussianSoA.from_scene(sc) for sc in frames]
    outs = [(torch.empty((c, H, W), device="cuda"), torch.empty((H, W), device="cuda"))
            for _ in frames]
    srv = Server(0, c=c, slots=1, max_batch=FRAMES, max_gauss_per_batch=FRAMES * n + 8192,
                 max_keys_per_batch=int(2.6 * FRAMES * n), max_pixels_per_batch=FRAMES * W * H,
                 max_side=max(W, H), keys_per_gaussian=2.5, batch_window_us=300000)
    torch.cuda.synchronize()
    tickets = [srv.submit(g, sc.cam, f, a, stream_id=k)
               for k, (sc, g, (f, a)) in enumerate(zip(frames, gs, outs))]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    assert all(r.status == 0 for r in results), [r.status for r in results]
    print("batch sizes", [r.batch_size for r in results], flush=True)
    assert max(r.batch_size for r in results) > 1

    rast = Rasterizer(0, max_n=n, max_w=W, max_h=H, keys_per_gaussian=2.5)
    for k, (sc, g, (fs, as_)) in enumerate(zip(frames, gs, outs)):
        print(f"[gpu] stress frame {k}: plain forward + backward", flush=True)
        feat, alpha = rast.forward(g, sc.cam)
        assert torch.equal(feat, fs) and torch.equal(alpha, as_), k
        T, last = rast.pixel_state(sc.cam)
        dF = scenes.make_cfg3_upstream(60 + k, c, H, W)
        gr = rast.backward(g, torch.as_tensor(dF, device="cuda"))
        torch.cuda.synchronize()
        got = {key: v.cpu().numpy() for key, v in gr.items()}
        gpu = dict(feat=feat.cpu().numpy(), alpha=alpha.cpu().numpy(), T=T.cpu().numpy(),
                   last=last.cpu().numpy())
        ora = oracle.Oracle(sc)
        ref_fwd = ora.render()
        rep = compare_forward(gpu, ora, ref=ref_fwd)
        worst, undet, loose = compare_backward(got, gpu, ora, dF, ref_fwd=ref_fwd)
        print(f"frame {k}", rep, "grads worst", worst, "undetermined pixels", undet,
              "loose Gaussians", loose, flush=True)
        ora.close()
