"""Host logic of the autotuner: tolerance selection and table lookup."""
import numpy as np

from paper_2110_03946_amd import autotune, synth


def _curve(rel, err, ms=None):
    ms = ms if ms is not None else [0.1 * (i + 1) for i in range(len(rel))]
    return np.array(rel), np.array(err), np.array(ms)


def test_pick_tol_largest_meeting_target():
    a = _curve([1e-2, 1e-3, 1e-4, 2e-5, 1e-5, 1e-5], [9, 2, 0.4, 0.2, 0.1, 0.1])
    b = _curve([2e-2, 2e-3, 3e-4, 5e-5, 1e-5, 1e-5], [9, 3, 0.6, 0.25, 0.1, 0.1])
    tol, cost, stops = autotune.pick_tol([a, b], target=0.3)
    # 1e-4 stops a at sweep 3 (0.4 > 0.3): too loose; 5e-5 stops a at 4
    # (0.2) and b at 4 (0.25)
    assert tol == 5e-5
    assert stops == [4, 4]
    assert abs(cost - 0.4) < 1e-12


def test_pick_tol_respects_min_sweeps_and_floor():
    # the first sweep already meets everything, but min_sweeps = 2
    a = _curve([1e-6, 5e-7, 1e-7, 1e-8], [0.1, 0.05, 0.03, 0.01])
    tol, _, stops = autotune.pick_tol([a], target=0.3, min_sweeps=2)
    assert stops == [2]
    # a floor at 4e-5 (no tolerance below 1.5x the floor is allowed)
    b = _curve([1e-3, 1e-4, 4e-5, 4e-5], [5, 1, 0.6, 0.6])
    assert autotune.pick_tol([b], target=0.3) is None


def test_sweep_floor():
    """The floor is the first sweep from which every image's error stays
    under the target to the end of its curve (a later rise moves it)."""
    a = _curve([1e-2, 1e-3, 1e-4, 1e-5], [2.0, 0.25, 0.2, 0.1])
    b = _curve([1e-2, 1e-3, 1e-4, 1e-5], [2.0, 0.4, 0.2, 0.1])
    assert autotune.sweep_floor([a], 0.3) == 2
    assert autotune.sweep_floor([a, b], 0.3) == 3
    c = _curve([1e-2, 1e-3, 1e-4, 1e-5], [0.2, 0.2, 0.35, 0.1])
    assert autotune.sweep_floor([c], 0.3) == 4
    assert autotune.sweep_floor([_curve([1e-2, 1e-3], [1.0, 0.9])], 0.3) is None
    # with min_sweeps at the floor, the tolerance is the loosest residual
    # every image meets from there: each stops at the floor
    tol, _, stops = autotune.pick_tol([a, b], 0.3, min_sweeps=3)
    assert tol == 1e-4 and stops == [3, 3]


def test_params_for_lookup():
    table = autotune.load_table()
    assert table["schedule"] == autotune.SCHEDULE
    assert len(table["classes"]) == len(synth.BATCH_SIZES) * len(autotune.KINDS) * \
        len(autotune.DENSITY_BUCKETS)
    for key, entry in table["classes"].items():
        p = entry["params"]
        for k, v in autotune.SCHEDULE.items():
            assert p[k] == v, key
        assert p["rel_tol"] > 0
        assert 0 <= p["overlap"] < p["block"] <= 64
        # the sweep floor measured for the class is its min_sweeps
        assert p["min_sweeps"] == entry["tuning"]["floor"] >= 1
    p = autotune.params_for(table, 2160, 3840, "clustered", 0.03)
    assert p == table["classes"]["2160x3840/clustered/0.02-0.05"]["params"]
    p = autotune.params_for(table, 1080, 1920, "bernoulli", 0.07)
    assert p == table["classes"]["1080x1920/bernoulli/0.05-0.10"]["params"]
    # an unseen size takes the nearest pixel count; a density outside the
    # buckets the nearest bucket
    p = autotune.params_for(table, 1000, 2000, "bernoulli", 0.15)
    assert p == table["classes"]["1080x1920/bernoulli/0.05-0.10"]["params"]


def test_batch_specs_recipe():
    specs = synth.batch_specs(48, 2)
    assert len(specs) == 48
    assert sum(s["kind"] == "clustered" for s in specs) == 24
    assert all((s["h"], s["w"]) in synth.BATCH_SIZES for s in specs)
    assert all(0.02 <= s["density"] <= 0.10 for s in specs)
    assert specs == synth.batch_specs(48, 2)


def test_widest_holes_picks_the_hardest_draws():
    """The tuning draws are those whose largest hole is widest: each picked
    mask's largest distance to a known pixel is at least that of every mask
    left out (checked by brute force on small masks)."""
    h, w, d = 40, 56, 0.03
    pick = autotune.widest_holes(h, w, "bernoulli", d, n_pick=4, n_draw=10)
    assert len(pick) == 4 and len(set(pick)) == 4

    def widest(i):
        c = synth.make_mask(h, w, d, "bernoulli", synth.mask_seed(autotune.TUNE_WORKLOAD, i))
        ky, kx = np.nonzero(c)
        yy, xx = np.mgrid[0:h, 0:w]
        dist = np.sqrt((yy[..., None] - ky) ** 2 + (xx[..., None] - kx) ** 2).min(axis=-1)
        return float(dist.max())

    scores = {i: widest(i) for i in range(10)}
    assert min(scores[i] for i in pick) >= max(scores[i] for i in range(10) if i not in pick)


def test_corner_hole():
    """The adversarial tuning mask: a quarter disk of 1.5 times the widest
    hole of the draws cleared at the top-left corner, the rest unchanged."""
    rng = np.random.default_rng(3)
    c = (rng.random((60, 80)) < 0.05).astype(np.uint8)
    out, r = autotune.corner_hole(c, [c])
    from scipy import ndimage
    widest = float(ndimage.distance_transform_edt(c == 0).max())
    assert abs(r - round(1.5 * widest, 1)) < 1e-9
    yy, xx = np.mgrid[0:60, 0:80]
    inside = yy * yy + xx * xx < (1.5 * widest) ** 2
    assert not out[inside].any()
    np.testing.assert_array_equal(out[~inside], c[~inside])
    # the corner hole is now the widest one
    assert ndimage.distance_transform_edt(out == 0).max() >= 1.5 * widest - 1
