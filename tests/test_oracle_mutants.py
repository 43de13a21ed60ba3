"""Plant plausible mistakes in a copy of the oracle and check the pins catch them.

Each mutant is one textual edit of ``oracle/fnr_oracle.c`` (a dropped term, a
wrong index or sign, a transposed operand, a misread of the paper), compiled to
a temporary library on the CPU.  A subset of the pins in ``test_oracle_pins.py``
runs against it and at least one must fail.  The unmutated source must pass
the same subset.  Every mutant keeps all memory accesses in bounds.
"""

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

MUTANTS = {
    # S_xy listing order: rows read bottom-up (the window as a set is unchanged)
    "window_rows_reversed": ("int yy = clamp_int(y + j, 0, H - 1);",
                             "int yy = clamp_int(y - j, 0, H - 1);"),
    # border reading: mirror instead of replicate at the left edge
    "border_mirror_left": ("int xx = clamp_int(x + i, 0, W - 1);",
                           "int xx = clamp_int(x + i < 0 ? -(x + i) : x + i, 0, W - 1);"),
    # window one row short
    "window_row_dropped": ("for (int j = -r; j <= r; ++j) {", "for (int j = -r; j < r; ++j) {"),
    # Step 2 tests only g_min
    "detector_min_only": ("return centre == gmin || centre == gmax;", "return centre == gmin;"),
    # Eq. 3a/3b scan drops the last window element
    "extreme_scan_short": ("for (int i = 1; i < n; ++i) {\n        if (S[i] > gmax)",
                           "for (int i = 1; i < n - 1; ++i) {\n        if (S[i] > gmax)"),
    # ties not flagged in flat windows (reading of Step 2 changed)
    "detector_strict_flat": ("return centre == gmin || centre == gmax;",
                             "return (centre == gmin || centre == gmax) && gmin != gmax;"),
    # median index one past the middle
    "median_index": ("return S[(n - 1) / 2];", "return S[(n + 1) / 2];"),
    # every pixel replaced (standard median filter instead of FNR)
    "replace_all": ("            if (replace) {\n                B[",
                    "            if (1) {\n                B["),
    # pass updates its own input in raster order instead of a snapshot
    "passes_in_place": ("uint64_t c = frame_pass(A, B, W, H, k, MODE_FNR",
                        "uint64_t c = frame_pass(A, A, W, H, k, MODE_FNR"),
    # insertion sort ordering reversed
    "insertion_descending": ("while (j >= 0 && a[j] > v) {", "while (j >= 0 && a[j] < v) {"),
    # heapsort picks the smaller child
    "heap_wrong_child": ("if (child + 1 < n && a[child + 1] > a[child]) child = child + 1;",
                         "if (child + 1 < n && a[child + 1] < a[child]) child = child + 1;"),
    # quicksort leaves the last element of the upper part unsorted
    "upper_part_short": ("introsort_range(a + cut, n - cut, depth, st); /* upper part */",
                         "insertion_sort(a + cut, n - cut - 1); /* upper part */"),
    # depth bound of zero: quicksort never runs (output unchanged, branch wrong)
    "depth_bound_zero": ("oracle_introsort_depth(a, n, n > 1 ? 2 * floor_log2(n) : 0, st);",
                         "oracle_introsort_depth(a, n, 0, st);"),
    # u16 pixels masked to 14 bits on read
    "u16_masked_14bit": ("                A[(size_t)y * W + x] = v;",
                         "                A[(size_t)y * W + x] = v & 0x3FFF;"),
}


def _run_pins():
    """The pin subset run against each build; raises AssertionError on a miss."""
    pins.test_window_listing_matches_paper_3x3_example()
    pins.test_window_border_replicates_edge_pixels()
    pins.test_table1_counts_every_pixel()
    for seed in range(12):
        pins.test_brute_force_tiny_frames(seed)
    pins.test_exhaustive_3x3_windows_over_three_levels()
    pins.test_two_dimensional_ramp_changes_only_at_its_extreme_corners()
    pins.test_constant_frame_is_fixed_point_with_every_pixel_flagged(3, "u8")
    for depth in (None, 0):
        pins.test_introsort_sorts(depth)
    pins.test_introsort_takes_the_quicksort_branch_for_windows_above_16()


def test_unmutated_source_passes_the_subset(tmp_path):
    lib = oracle.compile_source(oracle.source_text(), str(tmp_path / "orig.so"))
    with oracle.use_library(lib):
        _run_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    lib = oracle.compile_source(src.replace(old, new), str(tmp_path / f"{name}.so"))
    with oracle.use_library(lib):
        with pytest.raises(AssertionError):
            _run_pins()
