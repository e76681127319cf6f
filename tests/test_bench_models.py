"""The benchmark's FP64 operation count of the event-shape step, against an
independent tally of the same loop nests (pair scans written out as loops
over pairs rather than as closed forms)."""
import bench


def _tally(n):
    f = 0
    f += 13 * n  # validation: four sums, the mass shell and its tolerance per parton
    f += 25 * n + 15  # |p|, its reciprocal, the six tensor sums per parton; C
    f += 25 * n + 20  # hemisphere sums, masses and broadenings
    if n >= 3:
        for i in range(n):
            for j in range(i + 1, n):
                f += 9  # the plane's normal
                f += 9 * sum(1 for k in range(n) if k not in (i, j))  # signed sum of the others
                f += 4 * 12  # four sign choices of the pair
        f += 6  # thrust from the best plane
        f += 9 * n  # unit vectors for Durham
        m = n
        while m > 2:
            f += 13 * sum(1 for a in range(m) for b in range(a + 1, m))  # pair scan
            f += 13  # the merge
            m -= 1
    return f


def test_observable_flops_matches_the_loop_tally():
    for n in range(2, 40):
        assert bench.observable_flops(n) == _tally(n), n


def test_observable_flops_grows_like_n_cubed():
    # thrust's candidate planes dominate: n(n-1)/2 planes, n-2 partons each
    r = bench.observable_flops(200) / bench.observable_flops(100)
    assert 7.5 < r < 8.5
