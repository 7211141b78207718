"""Serving loop (paper_2110_03946_amd.serve) on small frames: every result
that reaches host memory is the inpainting of its request's frame (within
0.5 grey levels of the exact solution), slots stay within the HBM budget,
and requests wait in their queue when their class has no free slot."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_03946_amd import ddi, serve as mod
    ddi.lib()
    return mod


MIX = {(96, 128): 0.5, (130, 70): 0.3, (64, 200): 0.2}


@pytest.mark.parametrize("graph,realtime", [(True, False), (False, False), (True, True)])
def test_serve_results_and_admission(serve, graph, realtime):
    reqs, dens = serve.poisson_stream(400.0, 0.15, seed=9, mix=MIX, frames_per_size=2)
    pool = serve.frame_pool(dens, channels=3, workload=40)
    got = {}

    def keep(req, out):
        got[req.rid] = out.clone() if not out.is_cuda else out.cpu()

    # a budget of one slot per class: with all requests present at once the
    # queues must fill
    one = sum(serve.ddi.plan_footprint(h, w, 3, serve.ddi.default_params()) + 3 * h * w * 8 + h * w
              for (h, w) in MIX) * 2
    srv = serve.Server(channels=3, budget_bytes=int(one * 1.3), mix=MIX, use_graph=graph,
                       on_result=keep, max_slots=2)
    say("serve", len(reqs), "requests, graph", graph, "realtime", realtime, srv.stats.slots)
    srv.warmup(pool)
    st = srv.run(reqs, pool, realtime=realtime)
    srv.close()
    s = st.summary()
    say("  ", s)
    assert st.used_bytes <= st.budget_bytes
    assert len(got) == len(reqs) == s["requests"]
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    if not realtime:
        assert s["max_queue"] > 0
    exact = {}
    for r in reqs:
        f, c = pool[r.size][r.frame]
        key = (r.size, r.frame)
        if key not in exact:
            exact[key] = oracle.solve_exact(f.cpu().numpy().astype(np.float64), c.cpu().numpy())
        u = got[r.rid].numpy()
        assert np.abs(u - exact[key]).max() <= 0.5, r


def test_serve_hd_requests(serve):
    """720p and 1080p RGB requests through the serving loop with the tuned
    table (graph replays, results copied to host memory): every result within
    0.5 grey levels of the exact solution of its frame."""
    mix = {(720, 1280): 0.5, (1080, 1920): 0.5}
    reqs, dens = serve.poisson_stream(60.0, 0.4, seed=11, mix=mix, frames_per_size=1)
    pool = serve.frame_pool(dens, channels=3, workload=41)
    got = {}

    def keep(req, out):
        got[req.rid] = out.clone() if not out.is_cuda else out.cpu()

    srv = serve.Server(channels=3, budget_bytes=4 << 30, mix=mix, use_graph=True,
                       on_result=keep, max_slots=2)
    say("serve hd", len(reqs), "requests", srv.stats.slots)
    srv.warmup(pool)
    st = srv.run(reqs, pool, realtime=True)
    srv.close()
    say("  ", st.summary())
    assert len(got) == len(reqs) >= 10
    assert st.used_bytes <= st.budget_bytes
    exact = {}
    for r in reqs:
        f, c = pool[r.size][r.frame]
        key = (r.size, r.frame)
        if key not in exact:
            exact[key] = oracle.solve_exact(f.cpu().numpy().astype(np.float64), c.cpu().numpy())
        err = float(np.abs(got[r.rid].numpy() - exact[key]).max())
        assert err <= 0.5, (r.size, err)
