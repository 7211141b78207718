"""Host logic of the serving loop: the request stream."""
from paper_2110_03946_amd import serve


def test_poisson_stream_statistics():
    reqs, dens = serve.poisson_stream(120.0, 30.0, seed=4)
    assert abs(len(reqs) - 3600) < 4 * 60  # Poisson: sd = 60
    share = {s: sum(r.size == s for r in reqs) / len(reqs) for s in serve.SERVE_MIX}
    for s, p in serve.SERVE_MIX.items():
        assert abs(share[s] - p) < 0.03
    assert all(0.02 <= r.density <= 0.08 for r in reqs)
    assert all(a.arrival < b.arrival for a, b in zip(reqs, reqs[1:]))
