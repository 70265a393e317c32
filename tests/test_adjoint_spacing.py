"""The default snapshot spacing of FlameFront: the smallest K for which ceil(n / K)
snapshots plus a ring of K - 1 recomputed states fit the memory budget."""
from paper_2101_01702_amd.adjoint import snapshot_spacing


def test_every_state_when_they_fit():
    assert snapshot_spacing(4000, 1, 4000) == 1
    assert snapshot_spacing(4000, 2_200_000, 150e9) == 1


def test_smallest_spacing_that_fits():
    assert snapshot_spacing(4000, 1, 3999) == 2          # 2000 snapshots + a ring of 1
    assert snapshot_spacing(100, 1, 19) == 10            # 10 + 9; K = 9 needs 12 + 8
    for n, budget in [(4000, 150), (777, 60), (1, 5)]:
        k = snapshot_spacing(n, 1, budget)
        assert -(-n // k) + k - 1 <= budget
        assert k == 1 or -(-n // (k - 1)) + k - 2 > budget


def test_budget_below_any_spacing():
    assert snapshot_spacing(100, 10, 5) == 100
