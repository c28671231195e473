"""Write tests/golden/fixtures_sha256.json: SHA-256 of every array of the
workload generators' outputs (C0-C3, C5 and the first requests of C4), so that a
change to a generator or to the random streams it draws from shows up.

Calls only paper_2607_26901_amd.scenes (no oracle, no GPU code).
Run: python tests/golden/make_fixture_hashes.py"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2607_26901_amd import scenes as S  # noqa: E402

ARRAYS = ("x", "v", "inv_mass", "tris", "edges", "rest_x")
C4_FIRST = 16


def scene_hashes(sc):
    return {a: hashlib.sha256(getattr(sc, a).tobytes()).hexdigest() for a in ARRAYS}


def all_hashes():
    out = {name: scene_hashes(make()) for name, make in S.SCENES.items()}
    for rq in S.c4_requests()[:C4_FIRST]:
        out[f"c4_req{rq.rid}"] = dict(scene_hashes(rq.scene), arrival=repr(rq.arrival))
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "fixtures_sha256.json"), "w") as f:
        json.dump(all_hashes(), f, indent=1, sort_keys=True)
        f.write("\n")
