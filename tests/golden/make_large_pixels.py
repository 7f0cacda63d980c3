"""Writes large_pixels.json: the oracle's image of the large workload (100 x 100 x 120 A cell,
50,000 atoms, reflections to 1.5 A, 2048 x 2048 detector, Lorentzian 2 deg, Hosemann g .05
lateral, 96 x 96 nodes) at 1024 stratified pixels (tests/strata.py: 320 strong, 128 on the
meridian, 128 on the equator, 64 in the corners, 384 uniform), over the whole
extinction-culled reflection list with the oracle's own exact skip (oracle.reachable,
oracle.pattern_at), not over any culling list.

Calls only the oracle (oracle/), the seeded input generator (workloads/) and the pixel
strata (tests/strata.py, oracle only); nothing here touches the HIP library.  Run from the
repository root (about ten minutes on eight cores):

    python tests/golden/make_large_pixels.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402
from strata import stratified_pixels  # noqa: E402

OUT = os.path.join(HERE, "large_pixels.json")
COUNTS = {"strong": 320, "meridian": 128, "equator": 128, "corners": 64, "uniform": 384}
SEED = 2


def source_sha():
    """sha256 prefix of the oracle, input-generator and strata sources the values come from."""
    h = hashlib.sha256()
    for f in ("oracle/oracle.py", "oracle/oracle_c.c", "workloads/__init__.py", "tests/strata.py"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    t0 = time.time()
    wl = W.config2()
    hkl = O.enumerate_hkl(wl.cell, wl.quad.d_min, wl.quad.d_max)
    hkl = np.ascontiguousarray(hkl[~O.extinct_mask(hkl, wl.dis, wl.quad.extinction)])
    print(f"{hkl.shape[0]} reflections after the extinction cull; structure factors ({O.threads()} threads)", flush=True)
    F = O.structure_factors_c(hkl, wl.cell, wl.atoms)
    print(f"  {time.time() - t0:.0f} s", flush=True)
    P = O.prepare(wl, hkl=hkl, F=F, cull_extinct=False)
    pix = stratified_pixels(wl, P, COUNTS, SEED)
    q = np.array([p for p, _ in pix], dtype=np.int64)
    R, Z = O.pixel_rz(wl.geom)
    Rq, Zq = R.ravel()[q], Z.ravel()[q]
    sub = O.reachable(wl, hkl, Rq, Zq)
    print(f"{q.size} pixels reach {sub.size} reflections; pattern", flush=True)
    Ps = O.prepare(wl, hkl=np.ascontiguousarray(hkl[sub]), F=F[sub], cull_extinct=False)
    vals, n_ev = O.pattern_at(Ps, Rq, Zq, count=True)
    print(f"  {time.time() - t0:.0f} s, {n_ev} evaluations", flush=True)
    doc = {
        "what": "oracle image of the large workload at stratified pixels, all reflections, exact skip",
        "workload": wl.name,
        "script": "tests/golden/make_large_pixels.py",
        "sources_sha256_prefix": source_sha(),
        "strata_counts": COUNTS,
        "strata_seed": SEED,
        "n_hkl": int(hkl.shape[0]),
        "n_reachable": int(sub.size),
        "useful_evaluations": int(n_ev),
        "width": wl.geom.width,
        "height": wl.geom.height,
        "pixels": [{"q": int(p), "i": int(p % wl.geom.width), "j": int(p // wl.geom.width), "stratum": s,
                    "value": repr(float(v))} for (p, s), v in zip(pix, vals)],
    }
    with open(OUT + ".tmp", "w") as fh:
        json.dump(doc, fh, indent=0)
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} ({len(pix)} pixels) in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
