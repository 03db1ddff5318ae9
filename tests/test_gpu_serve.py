"""GPU tests of the serving loop (tg_serve_*): every request's result is the
same alone (plain path) and in the mix of a batch, the budget and the key
capacity are enforced, graph replay equals direct launches, and requests
submitted from several threads all complete."""
import threading

import numpy as np
import pytest

import oracle
import scenes
from gpu_common import compare_forward, torch_cuda

pytestmark = pytest.mark.gpu


def _requests(k=6, c=32, seed=100):
    """Uneven Gaussian counts, resolutions and poses (the serving generator,
    scaled down)."""
    out = []
    rng = np.random.default_rng(seed)
    for i in range(k):
        n = int(rng.integers(2000, 20000))
        res = int(rng.choice([64, 96, 128]))
        g = int(np.ceil(np.sqrt(n)))
        sc = scenes.make_grid_scene(seed + i, g, float(g), c, res, float(res),
                                    yaw=float(rng.uniform(-10, 10)), pitch=float(rng.uniform(-5, 5)), n=n)
        out.append(sc)
    return out


def _alone(scenes_, torch):
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    res = []
    for sc in scenes_:
        g = GaussianSoA.from_scene(sc)
        r = Rasterizer(0, max_n=sc.n, max_w=sc.cam.width, max_h=sc.cam.height)
        f, a = r.forward(g, sc.cam)
        res.append((f.cpu().numpy(), a.cpu().numpy()))
    return res


def _served(server, scenes_, torch, bg=None):
    """Submit every request back to back (inputs uploaded first), wait for all."""
    from paper_2405_14866_amd.rasterize import GaussianSoA
    gs = [GaussianSoA.from_scene(sc) for sc in scenes_]
    outs = [(torch.empty((sc.c, sc.cam.height, sc.cam.width), device="cuda"),
             torch.empty((sc.cam.height, sc.cam.width), device="cuda")) for sc in scenes_]
    torch.cuda.synchronize()
    tickets = [server.submit(g, sc.cam, f, a, bg=bg, stream_id=i % 3)
               for i, (sc, g, (f, a)) in enumerate(zip(scenes_, gs, outs))]
    results = [server.wait(t) for t in tickets]
    return [(f.cpu().numpy(), a.cpu().numpy()) for f, a in outs], results


@pytest.mark.parametrize("use_graph", [True, False])
def test_alone_equals_in_the_mix(use_graph):
    torch = torch_cuda()
    from paper_2405_14866_amd.serve import Server
    reqs = _requests()
    alone = _alone(reqs, torch)
    srv = Server(0, c=32, slots=2, max_batch=4, max_gauss_per_batch=60000, max_keys_per_batch=600000,
                 max_pixels_per_batch=4 * 128 * 128, max_side=128, use_graph=use_graph,
                 batch_window_us=200000)
    served, results = _served(srv, reqs, torch)
    srv.close()
    assert all(r.status == 0 for r in results), [r.status for r in results]
    assert max(r.batch_size for r in results) > 1          # requests were really batched
    for (fa, aa), (fs, as_) in zip(alone, served):
        # same kernels, same per-request lists: expected bitwise; the bar is the tolerance
        assert np.abs(fa - fs).max() <= 2e-4 and np.abs(aa - as_).max() <= 1e-5
    bitwise = all(np.array_equal(fa, fs) and np.array_equal(aa, as_) for (fa, aa), (fs, as_) in zip(alone, served))
    print("bitwise identical alone vs in the mix:", bitwise)
    assert bitwise


@pytest.mark.parametrize("c", [8, 64])
def test_served_request_matches_oracle(c):
    torch = torch_cuda()
    from paper_2405_14866_amd.serve import Server
    reqs = _requests(3, c=c, seed=300)
    bg = np.linspace(-1, 1, c).astype(np.float32)
    srv = Server(0, c=c, slots=1, max_batch=3, max_gauss_per_batch=60000, max_keys_per_batch=600000,
                 max_pixels_per_batch=3 * 128 * 128, max_side=128, batch_window_us=200000)
    served, results = _served(srv, reqs, torch, bg=torch.as_tensor(bg, device="cuda"))
    srv.close()
    assert results[0].batch_size == 3
    for sc, (f, a) in zip(reqs, served):
        ora = oracle.Oracle(sc)
        compare_forward(dict(feat=f, alpha=a, last=_last_placeholder(ora, sc, bg)), ora,
                        bg=bg.astype(np.float64), check_last=False)


def test_degenerate_requests_in_the_mix():
    """An empty request, one whose Gaussians are all behind the camera and
    one on a ragged 72x40 target, batched with two ordinary requests and a
    non-black background: every result equals its plain render bit for bit,
    the first two are the background with alpha 0, and the ragged one
    matches the oracle."""
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    from paper_2405_14866_amd.serve import Server
    c = 32
    cam = scenes.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 64.0, 64.0, 32.0, 32.0,
                        64, 64)
    empty = scenes.Scene(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((4, 0)), np.zeros(0),
                         np.zeros((0, c)), cam)
    behind = scenes.single_gaussian_scene(np.array([[0, 0, -1.0], [0, 0, 0.1]]).T, 0.05, c=c, cam=cam)
    body = scenes.make_body_scene(7, 48, 66.0, c, 72, 132.0)
    ragged = body.with_cam(scenes.Camera(body.cam.R, body.cam.t, body.cam.fx, body.cam.fy, 36.0, 20.0,
                                         72, 40))
    reqs = [_requests(1, c=c, seed=400)[0], empty, ragged, behind, _requests(1, c=c, seed=401)[0]]
    bg = np.linspace(-0.5, 0.5, c).astype(np.float32)
    bgt = torch.as_tensor(bg, device="cuda")
    plain = []
    for sc in reqs:
        r = Rasterizer(0, max_n=max(1, sc.n), max_w=sc.cam.width, max_h=sc.cam.height)
        f, a = r.forward(GaussianSoA.from_scene(sc), sc.cam, bgt)
        plain.append((f.cpu().numpy(), a.cpu().numpy()))
    srv = Server(0, c=c, slots=1, max_batch=len(reqs), max_gauss_per_batch=60000,
                 max_keys_per_batch=600000, max_pixels_per_batch=len(reqs) * 128 * 128, max_side=128,
                 batch_window_us=200000)
    served, results = _served(srv, reqs, torch, bg=bgt)
    srv.close()
    assert all(r.status == 0 for r in results), [r.status for r in results]
    print("batch sizes", [r.batch_size for r in results])
    assert max(r.batch_size for r in results) > 1
    for (fp, ap), (fs, as_) in zip(plain, served):
        assert np.array_equal(fp, fs) and np.array_equal(ap, as_)
    for k in (1, 3):
        f, a = served[k]
        assert np.all(a == 0)
        np.testing.assert_array_equal(f, np.broadcast_to(bg[:, None, None], f.shape))
    f, a = served[2]
    compare_forward(dict(feat=f, alpha=a), oracle.Oracle(ragged), bg=bg.astype(np.float64),
                    check_last=False)


def _last_placeholder(ora, sc, bg):
    return np.zeros((sc.cam.height, sc.cam.width), np.int32)


def test_budget_and_capacity():
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.rasterize import GaussianSoA
    from paper_2405_14866_amd.serve import Server
    reqs = _requests(4, seed=500)
    alone = _alone(reqs, torch)
    # a budget that holds the largest request alone: everything still completes, and
    # the requests in flight at any moment never exceed it (bytes a request occupies
    # in flight: padded state, estimated keys, pixel state and outputs)
    fp = lambda sc: (-(-sc.n // 1024) * 1024) * 76 + (int(sc.n * 5.0) + 1024) * 52 + \
        sc.cam.width * sc.cam.height * (8 + 4 * 33)
    budget = max(fp(sc) for sc in reqs)
    srv = Server(0, c=32, slots=2, max_batch=4, max_gauss_per_batch=60000, max_keys_per_batch=600000,
                 max_pixels_per_batch=4 * 128 * 128, max_side=128, budget_bytes=budget,
                 batch_window_us=100000)
    served, results = _served(srv, reqs, torch)
    assert all(r.status == 0 for r in results)
    assert sum(fp(sc) for sc in reqs) > budget            # the budget really limited the batches
    for i, (ri, si) in enumerate(zip(results, reqs)):
        # launched before, completed after ri's launch: in flight together with it
        live = fp(si) + sum(fp(sj) for j, (rj, sj) in enumerate(zip(results, reqs))
                            if j != i and rj.t_launch_ns <= ri.t_launch_ns < rj.t_done_ns)
        assert live <= budget, (i, live, budget)
    for (fa, aa), (fs, as_) in zip(alone, served):
        assert np.array_equal(fa, fs)
    # a request larger than the budget is refused at submit
    big = scenes.make_grid_scene(7, 200, 200.0, 32, 128, 128.0)
    g = GaussianSoA.from_scene(big)
    f = torch.empty((32, 128, 128), device="cuda")
    with pytest.raises(N.TgError) as ei:
        srv.submit(g, big.cam, f)
    assert ei.value.status == N.TG_ERR_BUDGET
    # a target larger than max_side is invalid
    cam = scenes.Camera(big.cam.R, big.cam.t, 64, 64, 64, 64, 256, 256)
    with pytest.raises(N.TgError):
        srv.submit(g, cam, torch.empty((32, 256, 256), device="cuda"))
    srv.close()


def test_wait_returns_when_another_caller_releases():
    """Two callers wait on one ticket and one of them releases it: both
    return (the other with the result or with TG_ERR_NOT_FOUND), none blocks."""
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.rasterize import GaussianSoA
    from paper_2405_14866_amd.serve import Server
    sc = _requests(1, seed=800)[0]
    srv = Server(0, c=32, slots=1, max_batch=1, max_gauss_per_batch=60000, max_keys_per_batch=600000,
                 max_pixels_per_batch=128 * 128, max_side=128)
    g = GaussianSoA.from_scene(sc)
    f = torch.empty((32, sc.cam.height, sc.cam.width), device="cuda")
    torch.cuda.synchronize()
    ticket = srv.submit(g, sc.cam, f)
    other = []
    th = threading.Thread(target=lambda: other.append(N.tg_serve_wait(srv.handle, ticket)[0]), daemon=True)
    th.start()
    res = srv.wait(ticket)                   # waits, then releases the ticket
    th.join(timeout=30)
    alive = th.is_alive()
    if not alive:
        srv.close()
    assert not alive, "the second waiter did not return"
    assert res.status == 0 and other[0] in (0, N.TG_ERR_NOT_FOUND), (res.status, other)


def test_key_overflow_is_readmitted_alone():
    """A batch that overflows the slot's key capacity is re-admitted one
    request at a time; a request that overflows alone fails."""
    torch = torch_cuda()
    from paper_2405_14866_amd.serve import Server
    reqs = _requests(3, seed=700)
    alone = _alone(reqs, torch)
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    nk = []
    for sc in reqs:
        r = Rasterizer(0, max_n=sc.n, max_w=sc.cam.width, max_h=sc.cam.height)
        r.forward(GaussianSoA.from_scene(sc), sc.cam)
        nk.append(r.n_keys)
    cap = max(nk) + 16                       # every request fits alone, the batch does not
    assert sum(nk) > cap
    srv = Server(0, c=32, slots=1, max_batch=3, max_gauss_per_batch=60000, max_keys_per_batch=cap,
                 max_pixels_per_batch=3 * 128 * 128, max_side=128, keys_per_gaussian=1e-3,
                 batch_window_us=200000)
    served, results = _served(srv, reqs, torch)
    assert results[0].batch_size == 1 and results[0].retries == 1
    assert all(r.status == 0 for r in results)
    assert any(r.retries > 0 for r in results)
    for (fa, aa), (fs, as_) in zip(alone, served):
        assert np.array_equal(fa, fs)
    srv.close()
    srv = Server(0, c=32, slots=1, max_batch=3, max_gauss_per_batch=60000, max_keys_per_batch=min(nk) // 2,
                 max_pixels_per_batch=3 * 128 * 128, max_side=128, keys_per_gaussian=1e-3)
    _, results = _served(srv, reqs[:1], torch)
    from paper_2405_14866_amd import _native as N
    assert results[0].status == N.TG_ERR_CAPACITY
    srv.close()


def test_threads_submit_concurrently():
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA
    from paper_2405_14866_amd.serve import Server
    reqs = _requests(8, c=16, seed=900)
    gs = [GaussianSoA.from_scene(sc) for sc in reqs]
    outs = [torch.empty((16, sc.cam.height, sc.cam.width), device="cuda") for sc in reqs]
    torch.cuda.synchronize()
    srv = Server(0, c=16, slots=3, max_batch=3, max_gauss_per_batch=60000, max_keys_per_batch=600000,
                 max_pixels_per_batch=3 * 128 * 128, max_side=128)
    tickets = [None] * len(reqs)

    def client(k):
        for i in range(k, len(reqs), 4):
            tickets[i] = srv.submit(gs[i], reqs[i].cam, outs[i], stream_id=k)

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    results = [srv.wait(t) for t in tickets]
    assert all(r.status == 0 for r in results)
    assert all(r.t_submit_ns <= r.t_launch_ns <= r.t_done_ns for r in results)
    srv.close()


def test_stream_arena_is_resident_and_budgeted():
    torch = torch_cuda()
    from paper_2405_14866_amd import _native as N
    from paper_2405_14866_amd.serve import Server
    srv = Server(0, c=8, slots=1, max_batch=2, max_gauss_per_batch=10000, max_keys_per_batch=100000,
                 max_pixels_per_batch=2 * 64 * 64, max_side=64, budget_bytes=4 << 20)
    a = srv.stream_arena(3, 5000)
    b = srv.stream_arena(3, 4000)
    assert a.mean and a.mean == b.mean and a.n == 5000 and a.c == 8
    with pytest.raises(N.TgError):
        srv.stream_arena(4, 1 << 20)         # would exceed the 4 MiB budget
    srv.close()


def test_serving_requests_at_full_size():
    """Six requests of the serving workload (100k..1M Gaussians each, C = 32,
    512^2..1024^2 targets) batched by the server: each equals its plain
    render bit for bit, and the smallest matches the oracle."""
    torch = torch_cuda()
    from paper_2405_14866_amd.serve import Server
    reqs = [scenes.make_cfg4_request(i) for i in range(6)]
    alone = _alone(reqs, torch)
    n_sum = sum(sc.n for sc in reqs)
    srv = Server(0, c=32, slots=2, max_batch=4, max_gauss_per_batch=n_sum + 8 * 1024,
                 max_keys_per_batch=int(4.0 * n_sum), max_pixels_per_batch=4 * 1024 * 1024,
                 max_side=1024, keys_per_gaussian=2.5, batch_window_us=300000)
    served, results = _served(srv, reqs, torch)
    srv.close()
    assert all(r.status == 0 for r in results), [r.status for r in results]
    assert max(r.batch_size for r in results) > 1
    for (fa, aa), (fs, as_) in zip(alone, served):
        assert np.array_equal(fa, fs) and np.array_equal(aa, as_)
    k = int(np.argmin([sc.n for sc in reqs]))
    ora = oracle.Oracle(reqs[k])
    f, a = served[k]
    rep = compare_forward(dict(feat=f, alpha=a, last=np.zeros_like(a, dtype=np.int32)), ora,
                          check_last=False)
    print("served request", k, reqs[k].n, rep)


def _plain_fwd_bwd(sc, dF, torch):
    """Plain frame-path forward and adjoint of one request (numpy outputs)."""
    from paper_2405_14866_amd.rasterize import GaussianSoA, Rasterizer
    g = GaussianSoA.from_scene(sc)
    r = Rasterizer(0, max_n=sc.n, max_w=sc.cam.width, max_h=sc.cam.height)
    f, a = r.forward(g, sc.cam)
    T, _ = r.pixel_state(sc.cam)
    gr = r.backward(g, torch.as_tensor(dF, device="cuda"))
    torch.cuda.synchronize()
    return f.cpu().numpy(), a.cpu().numpy(), {k: v.cpu().numpy() for k, v in gr.items()}, T.cpu().numpy()


def test_backward_in_the_loop_and_shared_sort():
    """Adjoints served in the batch, mixed with a forward-only request, and
    the reuse of an earlier request's projection and sorted lists: frame 1
    of stream 0 repeats frame 0's geometry (separate device copies, byte for
    byte equal) with new features and shares its sort; frame 2 of stream 0
    differs by one float in one mean and asks to share too, so the device
    check sends it back to render on its own.  Every image equals its plain
    render bit for bit; every gradient matches the plain adjoint within the
    gradient bar, and one shared request's gradients match the oracle."""
    torch = torch_cuda()
    from paper_2405_14866_amd.rasterize import GaussianSoA, empty_grads
    from paper_2405_14866_amd.serve import Server
    from gpu_common import compare_backward, compare_grads
    c = 32
    base, other, fwd_only = _requests(3, c=c, seed=500)
    rng = np.random.default_rng(501)
    f1 = (base.feat + 0.05 * rng.standard_normal(base.feat.shape)).astype(np.float32)
    frame1 = scenes.Scene(base.mean, base.scale, base.quat, base.opacity, f1, base.cam, name="frame1")
    mean2 = base.mean.copy()
    mean2[0, 17] = np.nextafter(mean2[0, 17], np.float32(1))
    frame2 = scenes.Scene(mean2, base.scale, base.quat, base.opacity, f1[::-1].copy(), base.cam, name="frame2")
    reqs = [(base, 0, True, False), (frame1, 0, True, True), (fwd_only, 1, False, False),
            (frame2, 0, True, True), (other, 2, True, False)]
    ups = [scenes.make_cfg3_upstream(510 + k, c, sc.cam.height, sc.cam.width) for k, (sc, *_r) in enumerate(reqs)]
    srv = Server(0, c=c, slots=1, max_batch=len(reqs), max_gauss_per_batch=120000, max_keys_per_batch=1200000,
                 max_pixels_per_batch=len(reqs) * 128 * 128, max_side=128, batch_window_us=300000,
                 backward=True)
    gs = [GaussianSoA.from_scene(sc) for sc, *_r in reqs]
    outs = [(torch.empty((c, sc.cam.height, sc.cam.width), device="cuda"),
             torch.empty((sc.cam.height, sc.cam.width), device="cuda")) for sc, *_r in reqs]
    grads = [empty_grads(sc.n, c) if bwd else None for sc, _s, bwd, _sh in reqs]
    dFs = [torch.as_tensor(u, device="cuda") for u in ups]
    torch.cuda.synchronize()
    print("[gpu] serve: adjoints in the loop, shared sort", flush=True)
    tickets = [srv.submit(g, sc.cam, f, a, stream_id=sid, d_feat=dF if bwd else None, grads=gr, share=sh)
               for (sc, sid, bwd, sh), g, (f, a), gr, dF in zip(reqs, gs, outs, grads, dFs)]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    assert all(r.status == 0 for r in results), [r.status for r in results]
    assert [r.shared for r in results] == [False, True, False, False, False], [r.shared for r in results]
    assert results[3].retries == 1 and results[1].retries == 0
    assert max(r.batch_size for r in results) >= 4
    for k, ((sc, _s, bwd, _sh), (f, a)) in enumerate(zip(reqs, outs)):
        pf, pa, pg, _ = _plain_fwd_bwd(sc, ups[k], torch)
        assert np.array_equal(f.cpu().numpy(), pf) and np.array_equal(a.cpu().numpy(), pa), k
        if bwd:
            got = {kk: v.cpu().numpy() for kk, v in grads[k].items()}
            compare_grads(got, pg, np.zeros(0, np.int64))
    # the shared request against the oracle's FP64 adjoint
    got = {kk: v.cpu().numpy() for kk, v in grads[1].items()}
    pf, pa, _, pT = _plain_fwd_bwd(frame1, ups[1], torch)
    ora = oracle.Oracle(frame1)
    ref = ora.render()
    gpu = dict(feat=pf, T=pT)
    print("shared request vs oracle", compare_backward(got, gpu, ora, ups[1], ref_fwd=ref))
