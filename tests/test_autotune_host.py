"""The tuned launch-shape table shipped with the package: every entry is a
shape the library accepts, keyed as the autotuner keys its sweeps."""
import json
import re

from paper_2511_11337_amd import autotune


def test_tuned_table_entries_are_valid_shapes():
    with open(autotune.TABLE) as fh:
        table = json.load(fh)
    assert table
    for key, shape in table.items():
        m = re.fullmatch(r"v3\|gfx\d+x\d+\|d(\d+)\|l(\d+)\|(f32|bf16|fp8)\|lanes(\d+)", key)
        assert m, key
        lanes = int(m.group(4))
        assert lanes & (lanes - 1) == 0, key                     # lane counts are rounded up to powers of two
        assert shape["tile_t"] in autotune.TILES, key
        assert shape["decode_kernel"] in ("fused", "steps"), key
        if shape["decode_kernel"] == "fused":
            assert shape["fused_lanes"] in autotune.FUSED_LANES, key
        assert isinstance(shape["use_graph"], bool), key
