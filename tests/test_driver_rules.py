"""Host rules of the multi-resolution driver (Algorithm 1): which decimation
levels take the far field and at what octree depth."""
from paper_2108_02991_amd import driver


def test_far_field_off_stays_exact():
    for d in range(7):
        assert driver._level_depth(0, d, 1 << 23) == 0


def test_small_levels_are_summed_exactly():
    # c3's coarsest level: 4096 shots x 32 samples
    assert driver._level_depth(5, 6, 4096 * 32) == 0
    assert driver._level_depth(5, 6, driver.EXACT_MAX_P) == 0
    assert driver._level_depth(5, 6, driver.EXACT_MAX_P + 1) == 3
    # with the threshold off, the depth rule alone decides
    assert driver._level_depth(5, 6, 4096 * 32, exact_max_p=0) == 3


def test_depth_drops_one_level_every_three_halvings():
    p = 1 << 23
    assert [driver._level_depth(5, d, p) for d in range(7)] == [5, 5, 4, 4, 4, 3, 3]
    assert [driver._level_depth(3, d, p) for d in range(7)] == [3, 3, 2, 2, 2, 0, 0]
