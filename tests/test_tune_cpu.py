"""Host logic of the launch-shape autotuner (no GPU)."""
import json

import pytest

from paper_2305_13555_amd import oci, tune


class _Ctx:
    n_angles, n_cells, n_regions = 32, 10000, 16
    precision = None


def test_fastest_prefers_the_smaller_shape_on_ties():
    assert tune.fastest({2: 1.0, 3: 0.5, 4: 0.7}) == 3
    assert tune.fastest({4: 0.5, 2: 0.5, 3: 0.9}) == 2


def test_cache_key_names_sizes_and_precision():
    c = _Ctx()
    assert tune.cache_key(c) == "N32_J10000_R16_fp64"
    c.precision = oci.OCI_PREC_FP32
    assert tune.cache_key(c) == "N32_J10000_R16_fp32"


def test_cache_round_trip(tmp_path):
    tune._cache.clear()
    tune._cache["N32_J10000_R16_fp64"] = 4
    path = tmp_path / "tune.json"
    tune.save_cache(str(path))
    tune._cache.clear()
    tune.load_cache(str(path))
    assert tune._cache == {"N32_J10000_R16_fp64": 4}
    path.write_text(json.dumps({"N8_J10_R1_fp64": 0}))
    with pytest.raises(ValueError):
        tune.load_cache(str(path))
    # the end-of-step fusion entries are 0 or 1
    tune._cache.clear()
    path.write_text(json.dumps({"N8_J10_R1_fp64_fusion": 0, "N8_J10_R1_fp32_fusion": 1}))
    tune.load_cache(str(path))
    assert tune._cache == {"N8_J10_R1_fp64_fusion": 0, "N8_J10_R1_fp32_fusion": 1}
    path.write_text(json.dumps({"N8_J10_R1_fp64_fusion": 2}))
    with pytest.raises(ValueError):
        tune.load_cache(str(path))
    tune._cache.clear()
