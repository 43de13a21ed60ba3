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
from tests import test_oracle_directional as dpins
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

# the opt-in directional detector (its own pins, test_oracle_directional.py)
DIRECTIONAL_MUTANTS = {
    # ties left out of the range (strict inequalities)
    "dir_strict_range": ("return lo <= c && c <= hi;", "return lo < c && c < hi;"),
    # noisy when non-monotone along any line instead of every line
    "dir_any_line": ("between(g, S[3], S[5]) || between(g, S[1], S[7]) ||",
                     "between(g, S[3], S[5]) && between(g, S[1], S[7]) &&"),
    # a diagonal paired with the wrong neighbour
    "dir_wrong_pair": ("between(g, S[0], S[8]) || between(g, S[2], S[6]);",
                       "between(g, S[0], S[2]) || between(g, S[6], S[8]);"),
    # the column line dropped
    "dir_column_dropped": ("between(g, S[3], S[5]) || between(g, S[1], S[7]) ||",
                           "between(g, S[3], S[5]) ||"),
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


def _run_directional_pins():
    for dt in (np.uint8, np.uint16):
        dpins.test_constant_frames_have_no_noise(dt)
    dpins.test_ramps_in_every_direction_have_no_noise()
    for val in (0, 255):
        dpins.test_interior_impulses_are_the_only_noise(val)
    dpins.test_one_pixel_lines_are_kept_while_the_extreme_detector_flags_them()
    dpins.test_border_pixels_are_never_noise()
    dpins.test_strict_extremes_are_noise_and_noise_differs_from_all_neighbours()
    for seed in range(6):
        dpins.test_dihedral_symmetry(seed)
    dpins.test_monotone_maps_and_complement_keep_the_flags()


def test_unmutated_source_passes_the_subset(tmp_path):
    lib = oracle.compile_source(oracle.source_text(), str(tmp_path / "orig.so"))
    with oracle.use_library(lib):
        _run_pins()
        _run_directional_pins()


@pytest.mark.parametrize("name", sorted(DIRECTIONAL_MUTANTS))
def test_directional_mutant_is_caught(name, tmp_path):
    old, new = DIRECTIONAL_MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    lib = oracle.compile_source(src.replace(old, new), str(tmp_path / f"{name}.so"))
    with oracle.use_library(lib):
        with pytest.raises(AssertionError):
            _run_directional_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    lib = oracle.compile_source(src.replace(old, new), str(tmp_path / f"{name}.so"))
    with oracle.use_library(lib):
        with pytest.raises(AssertionError):
            _run_pins()
