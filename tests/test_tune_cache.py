"""Host logic of the autotuner front end: cache keys and the JSON round trip
(no GPU needed; the library is loaded for its option defaults)."""
import json
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2602_12545_amd", "libfld.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfld.so not built")


def test_key_depends_on_shape_and_numerics_only():
    from paper_2602_12545_amd import tune, default_options
    a = default_options(precision="mixed")
    b = default_options(precision="mixed", smoother=1, chunk=4)   # tuned fields do not enter the key
    c = default_options(precision="fp64")
    assert tune._key("grid", [64, 32, 0], a) == tune._key("grid", [64, 32, 0], b)
    assert tune._key("grid", [64, 32, 0], a) != tune._key("grid", [64, 33, 0], a)
    assert tune._key("grid", [64, 32, 0], a) != tune._key("grid", [64, 32, 0], c)


def test_cache_round_trip(tmp_path):
    from paper_2602_12545_amd import tune, default_options
    path = str(tmp_path / "tune.json")
    base = default_options(precision="mixed", rel_tol=1e-11)
    tune._store(path, "k1", {"options": {"smoother": 2, "mg_coarse_max": 16, "chunk": 4}, "threads": 0, "ms": 1.5})
    tune._store(path, "k2", {"options": {"smoother": 1}, "threads": 256, "ms": 2.0})
    data = json.load(open(path))
    assert set(data) == {"k1", "k2"}
    o = tune._opt_from(data["k1"]["options"], base)
    assert (o.smoother, o.mg_coarse_max, o.chunk) == (2, 16, 4)
    assert o.precision == base.precision and o.rel_tol == base.rel_tol  # numerics kept from base
