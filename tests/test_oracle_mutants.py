"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks
that the oracle pins reject every one of them.

A starting value of 1 for the node-power loop is not planted: it is
equivalent, since floor(a) = floor(b) = 0 for midpoints in [0, 1)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    # merge takes from the right on ties (unstable)
    "unstable_merge": ("int take_right = (i >= mid) || (j < hi && less_at(A, j, i));",
                       "int take_right = (i >= mid) || (j < hi && !less_at(A, i, j));"),
    # weakly (not strictly) decreasing runs are reversed
    "nonstrict_descending_run": ("if (e < n && less_at(A, e, e - 1)) {\n        e++;  /* each adjacent pair is compared once */\n        while (e < n && less_at(A, e, e - 1)) e++;",
                                 "if (e < n && !less_at(A, e - 1, e)) {\n        e++;  /* each adjacent pair is compared once */\n        while (e < n && !less_at(A, e - 1, e)) e++;"),
    # midpoint without the half run length
    "midpoint_drops_half_length": ("unsigned __int128 an = 2 * (unsigned __int128)s1 + n1;",
                                   "unsigned __int128 an = 2 * (unsigned __int128)s1;"),
    # pops only on a power gap of two or more
    "stack_pop_condition": ("while (S->top > 0 && S->ps[S->top - 1] > p) {",
                            "while (S->top > 0 && S->ps[S->top - 1] > p + 1) {"),
    # min-run extension one element too long
    "min_run_off_by_one": ("uint64_t ew = (s + w < n) ? s + w : n;",
                           "uint64_t ew = (s + w + 1 < n) ? s + w + 1 : n;"),
    # insertion sort moves past equal keys
    "insertion_sort_unstable": ("while (j > s && key_less(A, v, A->key + (j - 1) * A->ks)) {",
                                "while (j > s && !key_less(A, A->key + (j - 1) * A->ks, v)) {"),
    # merge cost counts only the right run
    "merge_cost_right_only": ("S->M += hi - lo;", "S->M += hi - mid;"),
    # negative floats in increasing bit order
    "float_negative_order": ("return a > b;                 /* both negative",
                             "return a < b;                 /* both negative"),
    # midpoints of the wrong runs
    "power_swapped_runs": ("unsigned p = node_power(S->s1, S->e1 - S->s1, s2, e2 - s2, S->n);",
                           "unsigned p = node_power(S->s1, e2 - s2, s2, S->e1 - S->s1, S->n);"),
}

# Mistakes in the peeksort part, checked against the peeksort pins.
PEEK_MUTANTS = {
    # a tie between the two ends of the middle run goes to the left end
    "peek_tie_to_left": ("cut = (m - i < j - m) ? k : k + 1;", "cut = (m - i <= j - m) ? k : k + 1;"),
    # the farther end of the middle run
    "peek_far_end": ("cut = (m - i < j - m) ? k : k + 1;", "cut = (m - i < j - m) ? k + 1 : k;"),
    # the upper middle instead of the lower one
    "peek_midpoint_rounding": ("uint64_t m = l + (r - l) / 2;", "uint64_t m = l + (r - l + 1) / 2;"),
    # merge cost counts only the right part
    "peek_merge_cost_right_only": ("P->M += S[b] - S[a];", "P->M += S[b] - S[cut];"),
    # the right part's leaves one level too deep
    "peek_depth_off": ("peek_rec(P, cut, b, d + 1);", "peek_rec(P, cut, b, d + 2);"),
}


# Mistakes in the elementary mergesorts, checked against their pins.
MERGESORT_MUTANTS = {
    # the check merges runs that meet in equal keys (they are in order)
    "mergesort_check_nonstrict": ("    if (less_at(A, mid, mid - 1)) {  /* not already in order */",
                                  "    if (!less_at(A, mid - 1, mid)) {  /* not already in order */"),
    # the left half takes the floor of half the elements
    "topdown_split_floor": ("uint64_t mid = lo + (hi - lo + 1) / 2;", "uint64_t mid = lo + (hi - lo) / 2;"),
    # insertion sort only below w (pieces of exactly w are split once more)
    "topdown_cutoff_strict": ("    if (hi - lo <= w) {\n        insertion_sort(A, lo, hi, 0);",
                              "    if (hi - lo < w) {\n        insertion_sort(A, lo, hi, 0);"),
    # bottom-up run lengths start at 2w
    "bottomup_first_level_skipped": ("for (uint64_t m = w; m < n; m *= 2) {", "for (uint64_t m = 2 * w; m < n; m *= 2) {"),
}


# Mistakes in the galloping merge, checked against its pins.
GALLOP_MUTANTS = {
    # the right run's gallop also takes keys equal to the left head (ties go right)
    "gallop_right_nonstrict": (": key_less(A, A->key + (s + (k)) * A->ks, v))",
                               ": !key_less(A, v, A->key + (s + (k)) * A->ks))"),
    # the binary search after the exponential one skips the first candidate
    "gallop_binary_start": ("uint64_t a = lo + 1, b = (lo + hi < len) ? lo + hi : len;",
                            "uint64_t a = lo + 2, b = (lo + hi < len) ? lo + hi : len;"),
    # galloping mode is never entered
    "gallop_never": ("if (wins_left < kGallop && wins_right < kGallop) {", "if (1) {"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS) + sorted(PEEK_MUTANTS) + sorted(MERGESORT_MUTANTS)
                         + sorted(GALLOP_MUTANTS))
def test_pins_reject_planted_mistake(tmp_path, name):
    if name in MUTANTS:
        (a, b), suite = MUTANTS[name], "tests/test_oracle_pins.py"
    elif name in PEEK_MUTANTS:
        (a, b), suite = PEEK_MUTANTS[name], "tests/test_oracle_peeksort.py"
    elif name in MERGESORT_MUTANTS:
        (a, b), suite = MERGESORT_MUTANTS[name], "tests/test_oracle_mergesorts.py"
    else:
        (a, b), suite = GALLOP_MUTANTS[name], "tests/test_oracle_galloping.py"
    src = open(os.path.join(ROOT, "oracle", "powersort_oracle.c")).read()
    assert a in src, "mutation site not found"
    ign = shutil.ignore_patterns("*.so", "*.tmp", "__pycache__")
    for d in ("oracle", "tests", "paper_1805_04154_amd"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d, ignore=ign)
    (tmp_path / "oracle" / "powersort_oracle.c").write_text(src.replace(a, b))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        suite], cwd=tmp_path, capture_output=True, text=True,
                       timeout=600)
    # 1: a pin failed; a signal: the mutant crashed the suite (e.g. endless recursion)
    assert r.returncode == 1 or r.returncode < 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
