"""Host-side decoding of kbl_autotune_bounds' launch shapes (no device)."""

import paper_2407_20966_amd._lib as L


def test_decode_autotune_shapes():
    assert L.decode_autotune(8 * 12 + 0) == {"tile": 12, "elements_per_workgroup": 1}
    assert L.decode_autotune(8 * 3 + 2) == {"tile": 3, "workgroups_per_cu": 2}
    assert L.decode_autotune(8 * 5 + 5) == {"tile": 5, "elements_per_workgroup": 2}
    assert L.decode_autotune(6) == {"tile": 0, "elements_per_workgroup": 4}


def test_launch_workgroups():
    n_cu = 256
    assert L.launch_workgroups({"elements_per_workgroup": 1}, 1000, n_cu) == 1000
    assert L.launch_workgroups({"elements_per_workgroup": 2}, 2_000_000, n_cu) == 1_000_000
    # a multiple of 8 (one share per XCD), each share covering its range
    assert L.launch_workgroups({"elements_per_workgroup": 2}, 7, n_cu) == 8
    assert L.launch_workgroups({"elements_per_workgroup": 4}, 9, n_cu) == 8
    assert L.launch_workgroups({"elements_per_workgroup": 4}, 1_048_576, n_cu) == 262_144
    assert L.launch_workgroups({"workgroups_per_cu": 4}, 2_000_000, n_cu) == 1024
    assert L.launch_workgroups({"workgroups_per_cu": 8}, 100, n_cu) == 100


def test_shapes_match_the_header():
    text = open(L.HEADER).read()
    assert "5 = two and 6 = four elements per workgroup" in text
    assert len(L.AUTOTUNE_SHAPES) == 7
