"""Host logic of the training driver (no GPU): the learning-rate and batch
schedule of section 4 and the per-epoch permutations of a fixed data set."""
import pytest

from paper_2203_11025_amd import train


@pytest.mark.parametrize("epoch,changes", [(0, 0), (47, 0), (48, 1), (71, 1), (72, 2), (83, 2), (84, 3),
                                           (89, 3), (90, 4), (92, 4), (93, 5), (94, 5), (95, 6), (200, 6)])
def test_paper_schedule_change_epochs(epoch, changes):
    """Section 4: after t0 = 48 epochs the rate is divided by 10 and the batch
    doubled; further changes after t0 / 2^i more epochs (48, 72, 84, 90, ...)
    while that interval is at least one epoch."""
    lr, batch = train.paper_schedule(epoch, lr0=1e-4, batch0=20, t0=48)
    assert batch == 20 * 2 ** changes
    assert lr == pytest.approx(1e-4 / 10 ** changes, rel=1e-12)


def test_epoch_permutations_cover_the_data_set_once():
    b = train.Batches.__new__(train.Batches)
    b.dataset = 37
    for ep in range(3):
        idx = [b.index(5, ep * 37 + j) for j in range(37)]
        assert sorted(idx) == list(range(37))
    assert [b.index(5, j) for j in range(37)] != [b.index(5, 37 + j) for j in range(37)]
    b.dataset = None
    assert [b.index(5, j) for j in range(4)] == [0, 1, 2, 3]


def test_random_k_is_in_one_to_ten_and_reproducible():
    b = train.Batches.__new__(train.Batches)
    b.ksteps = "random"
    ks = [b.k_of(9, i) for i in range(2000)]
    assert set(ks) == set(range(1, 11))
    assert ks == [b.k_of(9, i) for i in range(2000)]
