"""The workload generators: every configuration starts valid (the paper states no
initial-intersection exclusion, so the minimum non-adjacent vertex-face,
edge-edge, particle-particle and particle-edge distance must be at least
xi + 0.1 mm), the strand generator's curl-halving rule fires where the
spacing clip alone would leave strands too close, and the generators
reproduce the recorded SHA-256 of
their arrays (tests/golden/fixtures_sha256.json, written by
tests/golden/make_fixture_hashes.py)."""
import json
import os

import numpy as np
import pytest

from paper_2607_26901_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _min_gap(orc, sc, need):
    xi = float(np.float32(sc.params.xi))
    d, below = orc.min_separation_grid(sc.x, sc.inv_mass, sc.tris, sc.edges, reach=4 * xi, below=need)
    return d, below


@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3", "c5"])
def test_workload_starts_valid(orc, name):
    sc = S.SCENES[name]()
    xi = float(np.float32(sc.params.xi))
    d, below = _min_gap(orc, sc, xi + 1e-4)
    assert below.sum() == 0 and d >= xi + 1e-4, (name, d, below)


def test_served_requests_start_valid(orc):
    reqs = S.c4_requests()
    # the smallest and largest cloths and a spread between
    sizes = np.array([r.scene.meta["cloth_n"] for r in reqs])
    pick = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes))] + list(range(0, 512, 73))))
    for i in pick:
        sc = reqs[i].scene
        xi = float(np.float32(sc.params.xi))
        d, below = _min_gap(orc, sc, xi + min(1e-4, 0.25 * xi))
        assert below.sum() == 0, (i, sc.name, d, below)


def test_strand_curl_halving_rule(orc):
    """Large curls with the spacing clip loosened threefold: the clip alone is
    not enough, the halving rule fires, and the strands start at least 2r + xi
    apart."""
    sc = S.helix_strands(n_strands=300, seg=32, curl=(15e-3, 20e-3), root_radius=0.04, seed=7,
                         root_spacing_scale=3.0)
    assert sc.meta["curl_halvings"] > 0
    band = 2 * float(np.float32(sc.params.r)) + float(np.float32(sc.params.xi))
    d, below = orc.min_separation_grid(sc.x, sc.inv_mass, sc.tris, sc.edges, reach=4 * band, below=band)
    assert below.sum() == 0 and d >= band, (d, below)
    # the default workload needs no halving
    assert S.c2().meta["curl_halvings"] == 0


def test_fixture_hashes():
    import hashlib
    want = json.load(open(os.path.join(GOLDEN, "fixtures_sha256.json")))
    for name, make in S.SCENES.items():
        sc = make()
        for a, h in want[name].items():
            assert hashlib.sha256(getattr(sc, a).tobytes()).hexdigest() == h, (name, a)
    reqs = S.c4_requests()
    for key, rec in want.items():
        if not key.startswith("c4_req"):
            continue
        rq = reqs[int(key[len("c4_req"):])]
        assert repr(rq.arrival) == rec["arrival"]
        for a in ("x", "v", "inv_mass", "tris", "edges", "rest_x"):
            assert hashlib.sha256(getattr(rq.scene, a).tobytes()).hexdigest() == rec[a], (key, a)
