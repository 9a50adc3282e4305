"""Host logic of the launch-shape tuner: size classes agree with the C header, and the committed
cache holds a compiled, accuracy-gated shape for every precision family and size class."""
import json
import os
import re

from paper_1003_3896_amd import autotune, nbody

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_size_classes_match_the_header():
    doc = open(os.path.join(ROOT, "include", "nbody.h")).read()
    line = re.search(r"nclass 0: largest cluster < (\d+) particles, 1: < (\d+), 2: < (\d+), 3: larger", doc)
    assert line, "size-class line of nbody_set_tile not found"
    b = [int(x) for x in line.groups()]
    assert len(b) + 1 == nbody.N_CLASSES
    for c, hi in enumerate(b):
        assert autotune.size_class(hi - 1) == c
        assert autotune.size_class(hi) == c + 1
    assert autotune.size_class(1) == 0
    assert autotune.size_class(1 << 30) == nbody.N_CLASSES - 1


def test_cache_covers_every_family_and_class_with_compiled_shapes():
    data = json.load(open(autotune.CACHE))
    for fam in ("f32", "ds", "f64", "dl"):
        for ncl in range(nbody.N_CLASSES):
            cfg = data["gfx950/%s/%d" % (fam, ncl)]
            kw = (cfg["k"], cfg["w"])
            assert kw in autotune.SHAPES, (fam, ncl, kw)
            if fam == "dl":
                assert kw not in autotune.NOT_DL
            assert cfg["tile"] in autotune.TILES
            assert 1 <= cfg["bpc"] <= 8
            if cfg["phase"]:
                assert fam in ("f32", "ds") and (cfg["k"], cfg["w"], cfg["tile"]) in autotune.PHASED
            prec = {"f32": "fp32c", "ds": "fp32ds", "f64": "fp64", "dl": "fp32dl"}[fam]
            assert cfg["err"] <= autotune.BOUND[prec][0]


def test_representative_workloads_fall_in_their_class():
    import numpy as np
    for ncl in range(nbody.N_CLASSES):
        b = autotune.representative(ncl)
        assert autotune.size_class(int(np.diff(b.offsets).max())) == ncl
