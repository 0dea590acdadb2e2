"""Pins of the fragmentation oracle (oracle.fragment) on configurations whose outcome follows from
the rules of the section "Fragmentation" by hand:

* a converging sphere (every particle reaches the peak at its own collapse time) is one halo;
* two such spheres far apart are two halos; spheres whose displaced centres meet merge when a
  particle touches both;
* a diverging sphere leaves a one-particle halo at the peak and filaments around it (case iv);
* invariants on random inputs: labels partition the collapsed particles, halo sizes count their
  members, a halo's id is a member (its founder), nothing below f_min is touched, and a periodic
  shift of the input shifts the partition.
"""

import numpy as np
import pytest

from oracle import fragment as FR

N = 16


def grid(n=N):
    i = np.arange(n ** 3)
    return np.stack([i // (n * n), (i // n) % n, i % n]).astype(np.float64)


def min_image(d, n=N):
    return d - n * np.floor(d / n + 0.5)


def sphere(center, f0=2.0, slope=0.02, sign=-1.0, n=N):
    """F peaked at `center` (decreasing with distance) and u = sign (q - c) F: with sign -1 each
    particle's displaced position q + u/F is exactly the centre."""
    q = grid(n)
    d = min_image(q - np.array(center, dtype=np.float64)[:, None], n)
    r2 = np.sum(d * d, axis=0)
    F = f0 - slope * r2
    u = sign * d * F
    return F, u


def flat_sigma(r):
    return 0.5


def test_converging_sphere_is_one_halo():
    F, u = sphere((8, 8, 8))
    f_min = 1.0
    label, sizes = FR.fragment(F, u, f_min, N, flat_sigma)
    collapsed = F >= f_min
    assert len(sizes) == 1
    h = next(iter(sizes))
    assert h == 8 * N * N + 8 * N + 8                 # founded by the peak
    assert np.all(label[collapsed] == h)
    assert np.all(label[~collapsed] == FR.NOT_COLLAPSED)
    assert sizes[h] == int(np.sum(collapsed))


def test_catalogue_of_a_converging_sphere():
    """One halo: its Lagrangian centre of mass is the peak (the members are symmetric about it) and
    its mean displacement vanishes (u is odd about the peak)."""
    F, u = sphere((8, 8, 8))
    label, sizes, (ids, cnt, centre, disp) = FR.fragment(F, u, 1.0, N, flat_sigma, catalog_cell=2.0)
    assert list(ids) == [8 * N * N + 8 * N + 8] and int(cnt[0]) == int(np.sum(F >= 1.0))
    assert np.allclose(centre[:, 0], 16.0, rtol=0, atol=1e-12)
    assert np.allclose(disp[:, 0], 0.0, rtol=0, atol=1e-12)


def test_catalogue_wraps_into_the_box():
    """A converging sphere centred on a corner: members on both sides of the periodic boundary, the
    centre of mass at the corner (0 after wrapping, not N/2)."""
    F, u = sphere((0, 0, 0))
    _, _, (ids, cnt, centre, _) = FR.fragment(F, u, 1.0, N, flat_sigma, catalog_cell=1.0)
    assert len(ids) == 1
    c = np.minimum(centre[:, 0], N - centre[:, 0])
    assert np.all(c <= 1e-12)


def test_merger_history_of_two_converging_peaks():
    """The two-peak case merges exactly once: the first halo (the higher peak founds it) keeps its
    id unless the other has grown larger, the sizes add up to the final halo, and the merger
    happens at the F of a particle touching both halos."""
    q = grid()
    c1, c2, mid = np.array([8.0, 6.0, 8.0]), np.array([8.0, 10.0, 8.0]), np.array([8.0, 8.0, 8.0])
    d1 = min_image(q - c1[:, None])
    d2 = min_image(q - c2[:, None])
    F = 2.0 - 0.05 * np.minimum(np.sum(d1 * d1, axis=0), np.sum(d2 * d2, axis=0) + 0.01)
    u = -min_image(q - mid[:, None]) * F
    label, sizes, mergers = FR.fragment(F, u, 1.2, N, flat_sigma, want_mergers=True)
    assert len(mergers) == 1
    f, keep, gone, nk, ng = mergers[0]
    assert {keep, gone} == {8 * N * N + 6 * N + 8, 8 * N * N + 10 * N + 8}
    assert nk >= ng and (nk > ng or keep < gone)
    assert sizes == {keep: sizes[keep]} and nk + ng <= sizes[keep]
    assert 1.2 <= f < 2.0


def test_no_mergers_for_distant_spheres():
    F1, u1 = sphere((4, 4, 4), f0=1.5, slope=0.1)
    F2, u2 = sphere((12, 12, 12), f0=1.4, slope=0.1)
    take = F1 >= F2
    _, _, mergers = FR.fragment(np.where(take, F1, F2), np.where(take[None], u1, u2), 1.0, N, flat_sigma,
                                want_mergers=True)
    assert mergers == []


def test_diverging_sphere_is_a_peak_and_filaments():
    F, u = sphere((8, 8, 8), sign=+1.0)
    label, sizes = FR.fragment(F, u, 1.0, N, flat_sigma)
    peak = 8 * N * N + 8 * N + 8
    assert sizes == {peak: 1}
    collapsed = F >= 1.0
    assert label[peak] == peak
    rest = collapsed.copy()
    rest[peak] = False
    assert np.all(label[rest] == FR.FILAMENT)


def test_two_distant_spheres_are_two_halos():
    F1, u1 = sphere((4, 4, 4), f0=1.5, slope=0.1)
    F2, u2 = sphere((12, 12, 12), f0=1.4, slope=0.1)
    take = F1 >= F2
    F = np.where(take, F1, F2)
    u = np.where(take[None], u1, u2)
    label, sizes = FR.fragment(F, u, 1.0, N, flat_sigma)
    a, b = 4 * N * N + 4 * N + 4, 12 * N * N + 12 * N + 12
    assert set(sizes) == {a, b}
    assert np.all(label[(F1 >= 1.0) & take] == a)
    assert np.all(label[(F2 >= 1.0) & ~take] == b)


def test_touching_spheres_with_a_common_centre_merge():
    """Two peaks 4 cells apart whose particles all converge on the midpoint: the two halos touch
    once they grow, their displaced centres coincide, and they merge into one."""
    q = grid()
    c1, c2, mid = np.array([8.0, 6.0, 8.0]), np.array([8.0, 10.0, 8.0]), np.array([8.0, 8.0, 8.0])
    d1 = min_image(q - c1[:, None])
    d2 = min_image(q - c2[:, None])
    F = 2.0 - 0.05 * np.minimum(np.sum(d1 * d1, axis=0), np.sum(d2 * d2, axis=0) + 0.01)
    u = -min_image(q - mid[:, None]) * F                      # every particle reaches the midpoint
    label, sizes = FR.fragment(F, u, 1.2, N, flat_sigma)
    collapsed = F >= 1.2
    assert len(sizes) == 1
    h = next(iter(sizes))
    assert np.all(label[collapsed] == h) and sizes[h] == int(np.sum(collapsed))


def random_inputs(seed, n=N, f_hi=3.0):
    rng = np.random.default_rng(seed)
    # a smooth random F (sum of a few waves) so that halos and filaments both occur
    q = grid(n)
    F = np.full(n ** 3, 1.0)
    for _ in range(6):
        k = rng.integers(-2, 3, 3)
        F += 0.4 * np.cos(2 * np.pi * (k @ q) / n + rng.uniform(0, 2 * np.pi))
    F += 1e-6 * rng.standard_normal(n ** 3)                   # no ties
    u = -0.8 * np.stack([np.sin(2 * np.pi * q[a] / n + rng.uniform(0, 6.3)) for a in range(3)]) * n / 8
    return np.clip(F, 0.0, f_hi), u


@pytest.mark.parametrize("seed", [1, 2])
def test_invariants_on_random_inputs(seed):
    F, u = random_inputs(seed)
    f_min = 1.2
    label, sizes = FR.fragment(F, u, f_min, N, flat_sigma)
    collapsed = F >= f_min
    assert np.all(label[~collapsed] == FR.NOT_COLLAPSED)
    assert np.all(label[collapsed] != FR.NOT_COLLAPSED)
    assert len(sizes) > 1 and np.any(label == FR.FILAMENT)
    for h, s in sizes.items():
        assert label[h] == h
        assert int(np.sum(label == h)) == s
    assert sum(sizes.values()) == int(np.sum(label >= 0))


def test_periodic_shift_shifts_the_partition():
    F, u = random_inputs(3)
    f_min = 1.2
    label, _ = FR.fragment(F, u, f_min, N, flat_sigma)
    sh = (5, 3, 11)
    Fs = np.roll(F.reshape(N, N, N), sh, axis=(0, 1, 2)).ravel()
    us = np.stack([np.roll(u[a].reshape(N, N, N), sh, axis=(0, 1, 2)).ravel() for a in range(3)])
    label_s, _ = FR.fragment(Fs, us, f_min, N, flat_sigma)
    back = np.roll(label_s.reshape(N, N, N), tuple(-s for s in sh), axis=(0, 1, 2)).ravel()
    # same classes: NOT_COLLAPSED and FILAMENT exactly, halos as a partition (ids move)
    assert np.array_equal(back < 0, label < 0) and np.array_equal(back[back < 0], label[label < 0])
    pairs = {}
    for a, b in zip(label[label >= 0], back[label >= 0]):
        assert pairs.setdefault(a, b) == b
    assert len(set(pairs.values())) == len(pairs)


def test_sigma_table():
    from oracle import spectrum

    n, box = 64, 128.0
    t = FR.SigmaTable(n, box, 0.8, 0.21, 1.0, nh_max=10 ** 5)
    # exact at the nodes, and sigma at the radius of 8 Mpc/h is sigma8 within interpolation error
    r = t.r0 * 2.0 ** (10 / 64)
    amp = spectrum.amplitude_for_sigma8(0.8, 0.21, 1.0)
    # the table's Simpson rule against the adaptive quadrature
    assert abs(t(r) / np.sqrt(spectrum.sigma2_tophat(r * box / n, 0.21, 1.0, amp)) - 1.0) <= 1e-10
    assert abs(t(8.0 * n / box) - 0.8) <= 1e-4
    assert t(1.0) > t(2.0) > t(4.0)
