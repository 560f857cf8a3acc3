"""Plant plausible mistakes in the oracle (on the CPU, by monkeypatching)
and check that at least one pin fails for each: a pin that cannot fail
pins nothing."""
import numpy as np
import pytest

from oracle import mask_oracle as mo
from tests import test_oracle_pins as pins


def _fails(fn):
    try:
        fn()
    except AssertionError:
        return True
    return False


def test_wrong_sign_in_distance_is_caught(monkeypatch):
    orig = mo.pairwise

    def bad(A, B, metric="l2", block=256):
        return orig(A, -np.asarray(B), metric, block)
    monkeypatch.setattr(mo, "pairwise", bad)
    assert _fails(pins.test_assign_matches_brute_force_loops)


def test_dropped_dimension_is_caught(monkeypatch):
    orig = mo.pairwise

    def bad(A, B, metric="l2", block=256):
        return orig(np.asarray(A)[:, 1:], np.asarray(B)[:, 1:], metric, block)
    monkeypatch.setattr(mo, "pairwise", bad)
    assert _fails(pins.test_probe_all_is_exact_knn)


def test_biased_mean_is_caught(monkeypatch):
    orig = mo.update

    def bad(points, labels, centroids, metric="l2"):
        new, counts = orig(points, labels, centroids, metric)
        return new * (1 + 1e-6), counts
    monkeypatch.setattr(mo, "update", bad)
    assert _fails(pins.test_kmeans_one_prototype_is_the_mean)
    assert _fails(pins.test_kmeans_matches_scipy_kmeans2_with_given_init)


def test_empty_prototype_reset_is_caught(monkeypatch):
    orig = mo.update

    def bad(points, labels, centroids, metric="l2"):
        new, counts = orig(points, labels, centroids, metric)
        new[counts == 0] = 0.0
        return new, counts
    monkeypatch.setattr(mo, "update", bad)
    assert _fails(pins.test_empty_prototype_keeps_its_value)


def test_upper_median_is_caught(monkeypatch):
    monkeypatch.setattr(mo, "lower_median",
                        lambda v: np.sort(v, axis=0)[v.shape[0] // 2])
    assert _fails(pins.test_lower_median_minimises_l1_and_is_a_data_value)


def test_farthest_selection_is_caught(monkeypatch):
    monkeypatch.setattr(mo, "smallest", lambda d, ids, m: np.lexsort((ids, -d))[:m])
    assert _fails(pins.test_greedy_descent_follows_nearest_prototype)


def test_transposed_chunking_is_caught(monkeypatch):
    # groups taken as strided instead of contiguous slices
    def bad(n_items, n_chunks):
        off = np.zeros(n_chunks + 1, dtype=np.int64)
        off[1:] = np.arange(1, n_chunks + 1) * (n_items // n_chunks)
        off[-1] = n_items
        return off
    monkeypatch.setattr(mo, "chunk_offsets", bad)
    assert _fails(pins.test_chunk_offsets_match_numpy_array_split)


def test_off_by_one_schedule_is_caught(monkeypatch):
    # stops while one full group is still left (">" instead of ">=")
    def bad(n, lg, nc):
        levels, ng = [], n // lg
        while ng > 1:
            levels.append((ng, nc))
            ng = (ng * nc) // lg
        return levels
    monkeypatch.setattr(mo, "plan_levels", bad)
    assert _fails(pins.test_level_schedule_tree_depths)


def test_wrong_splitmix_constant_is_caught(monkeypatch):
    monkeypatch.setattr(mo, "_M2", np.uint64(0x94D049BB133111EA))
    assert _fails(pins.test_splitmix64_known_answers)


def test_range_radius_not_squared_is_caught(monkeypatch):
    # comparing squared distances with the radius itself (not its square)
    orig = mo.range_query_one

    def bad(index, q, radius, max_out, level_cap):
        return orig(index, q, float(radius) ** 0.5, max_out, level_cap)
    monkeypatch.setattr(mo, "range_query_one", bad)
    assert _fails(pins.test_range_search_on_one_to_one_index_is_exact)


def test_range_strict_boundary_drops_the_exact_match(monkeypatch):
    # a strict "<" at the boundary would lose the point at radius 0
    orig_pairwise = mo.pairwise

    def bad(A, B, metric="l2", block=256):
        return orig_pairwise(A, B, metric, block) + 1e-300
    monkeypatch.setattr(mo, "pairwise", bad)
    assert _fails(pins.test_range_search_on_one_to_one_index_is_exact)


def test_point_query_on_the_wrong_level_is_caught(monkeypatch):
    # children taken one level too low on the way down
    orig = mo.OracleIndex.children

    def bad(self, level):
        return orig(self, max(level - 1, 0))
    monkeypatch.setattr(mo.OracleIndex, "children", bad)
    with pytest.raises((AssertionError, IndexError)):
        pins.test_point_query_is_the_greedy_descent_then_a_leaf_scan()


def test_point_query_answering_with_the_farthest_point_is_caught(monkeypatch):
    orig = mo.pairwise

    def bad(A, B, metric="l2", block=256):
        return -orig(A, B, metric, block)
    monkeypatch.setattr(mo, "pairwise", bad)
    assert _fails(pins.test_point_query_on_one_to_one_level_finds_every_point)


# ---------------------------------------------------- comparator and replay

from oracle import compare as oc  # noqa: E402


def test_selection_check_that_accepts_anything_is_caught(monkeypatch):
    monkeypatch.setattr(oc, "check_selection", lambda *a, **k: None)
    assert _fails(pins.test_check_selection_accepts_nearest_sets_and_near_ties_only)
    assert _fails(pins.test_replay_follows_a_tied_selection_and_rejects_a_farther_one)


def test_selection_check_without_a_tie_band_is_caught(monkeypatch):
    orig = oc.check_selection

    def strict(cand, cand_dist, sel, r, rel=1e-5, abs_tol=0.0):
        return orig(cand, cand_dist, sel, r, 0.0, 0.0)
    monkeypatch.setattr(oc, "check_selection", strict)
    assert _fails(pins.test_check_selection_accepts_nearest_sets_and_near_ties_only)


def test_replay_that_ignores_the_forced_selection_is_caught(monkeypatch):
    orig = mo.query_one

    def bad(index, q, k, r, trace=False, forced=None):
        return orig(index, q, k, r, trace=trace)
    monkeypatch.setattr(mo, "query_one", bad)
    assert _fails(pins.test_replay_follows_a_tied_selection_and_rejects_a_farther_one)


def test_rerank_check_without_the_low_precision_cut_is_caught(monkeypatch):
    orig = oc.check_rerank

    def bad(got_ids, got_dist, cand, d_low, d_full, k, R, rel=1e-5):
        return orig(got_ids, got_dist, cand, d_low, d_full, k, 10 ** 9, rel)
    monkeypatch.setattr(oc, "check_rerank", bad)
    assert _fails(pins.test_check_rerank_takes_the_low_precision_cut_then_the_full_ranking)


# ----------------------------------------------------------- precision form

def test_truncating_bf16_is_caught(monkeypatch):
    def trunc(X):
        x = np.ascontiguousarray(X, dtype=np.float32)
        u = x.view(np.uint32) & np.uint32(0xFFFF0000)
        return u.view(np.float32).astype(np.float64)
    monkeypatch.setattr(mo, "quantize_bf16", trunc)
    assert _fails(pins.test_bf16_rounding_matches_torch_and_ties_to_even)


def test_e4m3_rounding_half_away_from_zero_is_caught(monkeypatch):
    def away(v):
        v = np.asarray(v, dtype=np.float64)
        a = np.abs(v)
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
        step = np.where(a >= 2.0 ** -6, 2.0 ** (e - 3), 2.0 ** -9)
        return np.sign(v) * np.floor(a / step + 0.5) * step
    monkeypatch.setattr(mo, "round_e4m3", away)
    assert _fails(pins.test_e4m3_rounding_matches_torch_and_keeps_every_code)


def test_fp8_scale_off_by_one_step_is_caught(monkeypatch):
    orig = mo.quantize_fp8

    def bad(X):
        code, s = orig(X)
        return code, s * (1 + 2.0 ** -3)
    monkeypatch.setattr(mo, "quantize_fp8", bad)
    assert _fails(pins.test_fp8_rows_reconstruct_within_half_a_step)


def test_preselection_on_the_full_rows_is_caught(monkeypatch):
    orig = mo.query_one_lowp

    def bad(index, q, k, r, rank_protos, leaf_rows, factor, forced=None, trace=False):
        return orig(index, q, k, r, rank_protos, index.data, factor, forced, trace)
    monkeypatch.setattr(mo, "query_one_lowp", bad)
    assert _fails(pins.test_lowp_descent_preselects_by_the_low_precision_rows)


def test_rerank_cap_ignoring_the_beams_is_caught(monkeypatch):
    monkeypatch.setattr(mo, "rerank_size", lambda k, beams, factor: min(factor * k, 512))
    assert _fails(pins.test_rerank_size_caps)


def test_screened_bound_without_the_query_split_term_is_caught(monkeypatch):
    def bad(q, rows):
        q = np.asarray(q, dtype=np.float64)
        cmax = float(np.einsum("ij,ij->i", rows, rows).max())
        return 2.0 ** -24 * (float(q @ q) + cmax)
    monkeypatch.setattr(oc, "screened_bound", bad)
    assert _fails(pins.test_screened_bound_covers_the_float32_expanded_form)


def test_rerank_cap_from_k_and_beams_only_is_caught(monkeypatch):
    # the cap must also rise when the set itself passes 512
    def bad(k, beams, factor):
        cap = 512 if max([k] + list(beams)) <= 512 else 2048
        r0 = -factor * k * beams[-1] if factor < 0 else factor * k
        return min(r0, cap)
    monkeypatch.setattr(mo, "rerank_size", bad)
    assert _fails(pins.test_rerank_size_caps)


def test_rerank_set_without_the_leaf_beam_is_caught(monkeypatch):
    monkeypatch.setattr(mo, "rerank_size",
                        lambda k, beams, factor: min(abs(factor) * k, 2048))
    assert _fails(pins.test_rerank_size_caps)
