"""Host logic of bench.py that the reported work and rooflines rest on: the changed
pairs a schedule fixes (closed forms of the rigid-body fact, and brute force over
pairs and tiles), and the source digest that ties the counter record to the code."""
import os

import pytest

import bench


def _changed_pairs_brute(L, k, h=None):
    """Pairs i < j whose distance changes when torsion k turns (one side of the
    pivot moves rigidly), optionally only inside the window [c - h, c + h]."""
    c = k // 2
    p = c + 1 if k % 2 else c
    lo, hi = (0, L - 1) if h is None else (max(0, c - h), min(L - 1, c + h))
    return sum(1 for i in range(lo, hi + 1) for j in range(i + 1, hi + 1) if i < p <= j)


@pytest.mark.parametrize("L", [2, 3, 17, 64, 300])
def test_global_sweep_pairs_closed_form(L):
    """A global sweep changes sum_k p_k (L - p_k) = (L^3 - L) / 3 pairs: 87,360 at
    L = 64 and 8,999,900 at L = 300."""
    glob, _ = bench.pair_evals_per_cycle(L, 12, 10)
    assert glob == (L ** 3 - L) // 3
    if L <= 64:
        assert glob == sum(_changed_pairs_brute(L, k) for k in range(2 * L))
    assert bench.pair_evals_per_cycle(64, 8, 10)[0] == 87360
    assert bench.pair_evals_per_cycle(300, 12, 10)[0] == 8999900


@pytest.mark.parametrize("L,d", [(2, 2), (10, 4), (40, 8), (64, 12), (33, 64)])
def test_local_sweep_pairs_brute_force(L, d):
    """Localized pairs per cycle (cycle - 1 localized sweeps): every proposal's
    changed pairs inside its window, h (h + 1) in the interior."""
    h = d // 2
    per_sweep = sum(_changed_pairs_brute(L, k, h) for k in range(2 * L))
    for cycle in (1, 2, 10):
        assert bench.pair_evals_per_cycle(L, d, cycle)[1] == per_sweep * (cycle - 1)
    if L > 2 * h + 2:
        k = 2 * (h + 1)   # phi of an interior residue, and the psi after it
        assert _changed_pairs_brute(L, k, h) == h * (h + 1)
        assert _changed_pairs_brute(L, k + 1, h) == h * (h + 1)


@pytest.mark.parametrize("L", [2, 9, 40, 300])
def test_candidate_tiles_brute_force(L):
    """Candidate 8 x 8 tiles of the global rectangles: every (row block, column block)
    holding at least one pair i < p <= j with i, j < L, summed over the proposals."""
    nb8 = (L + 7) // 8
    brute = 0
    for k in range(2 * L):
        p = (k + 1) // 2
        for I in range(nb8):
            for J in range(nb8):
                rows = range(8 * I, min(8 * I + 8, L))
                cols = range(8 * J, min(8 * J + 8, L))
                if any(i < p <= j for i in rows for j in cols):
                    brute += 1
    work = bench.schedule_work(L, 12, 10)
    assert work["candidate_tiles"] == brute
    assert work["transition_pairs"] == L * (L - 1)
    assert work["anchor_pairs"] == L * (L - 1) // 2


def test_code_digest_follows_code_not_comments(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one\n}\n/* block */\n")
    d0 = bench.code_digest(["a.hip"])
    a.write_text("int f(int x) { return x + 1; }  // another comment\n")
    assert bench.code_digest(["a.hip"]) == d0
    a.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_digest(["a.hip"]) != d0


def test_committed_counter_record_matches_the_sources():
    """The HBM byte record used for the benchmark's traffic field was taken on the
    committed kernel sources (else the benchmark reports traffic as null)."""
    assert os.path.exists(bench.TRAFFIC_RECORD)
    t = bench.measured_traffic()
    assert t is not None and t["local"] > 0 and t["global"] > 0
