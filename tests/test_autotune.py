"""The tuner's table arithmetic (no GPU): key widths, and the rows written for
tuned list sizes (ascending, each applying from the geometric middle between
its size and the previous one)."""
import json

from paper_1802_05931_amd import autotune


def test_key_bytes():
    assert autotune.key_bytes(16) == 4      # 4x4 alone: 32 bits
    assert autotune.key_bytes(25) == 8      # 5x5: 50 bits
    assert autotune.key_bytes(16, 64) == 8  # a 64-slot pool of 4x4: 38 bits
    assert autotune.key_bytes(9, 64) == 4   # 3x3 in 64 slots: 24 bits
    assert autotune.key_bytes(25, 64) == 8  # 5x5 in 64 slots: 56 bits


def test_table_rows(tmp_path):
    runs = [dict(label="a", key_bytes=4, n_entries=10_000_000, sort_it=8, merge_it=8, ms={}),
            dict(label="b", key_bytes=4, n_entries=100_000, sort_it=4, merge_it=4, ms={}),
            dict(label="c", key_bytes=8, n_entries=4_000_000, sort_it=16, merge_it=8, ms={})]
    p = tmp_path / "t.json"
    out = autotune.write_table(runs, str(p))
    assert out["rows"]["k4"] == [[0, 4, 4], [1_000_000, 8, 8]]
    assert out["rows"]["k8"] == [[0, 16, 8]]
    assert json.load(open(p))["runs"] == runs

    class H:
        def set_tile_table(self, rows):
            self.rows = rows
    h = H()
    assert autotune.apply(h, 4, str(p)) == [[0, 4, 4], [1_000_000, 8, 8]]
    assert h.rows == [(0, 4, 4), (1_000_000, 8, 8)]
    assert autotune.apply(H(), 4, str(tmp_path / "missing.json")) == []
