"""The plateau sector analysis of the learned-MH comparison (host code, no
GPU): an ordered state at the plateau's magnetisation and wavevector has
O_1/3 = 1/3 exactly, lattice
translations by two columns and the transpose move it to another sector,
maps onto itself are no move, and disordered states never count."""
import numpy as np

from paper_2511_20911_amd import learned

L = 18


def _ordered(L=L):
    """Period-3 stripes of down spins along the columns, shifted by two
    columns on odd rows: S_A = (-2 L / 3)(L / 2)(1 - w^2), w = e^{2 pi i / 3},
    so |S_A|^2 / N^2 = 1/3."""
    s = np.ones((L, L), dtype=np.int8)
    for r in range(L):
        k = 0 if r % 2 == 0 else 2
        s[r, k::3] = -1
    return s


def _sectors(*states):
    return learned.plateau_sectors(np.stack(states))


def test_ordered_state_has_the_plateau_order_parameter():
    s = _ordered()
    o, ph, ok = _sectors(s)
    c = np.arange(L)[None, :]
    r = np.arange(L)[:, None]
    sa = np.sum(s * np.exp(1j * (np.pi * r + 2 * np.pi * c / 3)))
    assert abs(abs(sa) ** 2 / L ** 4 - 1.0 / 3.0) < 1e-12
    assert o[0] == 0 and ok[0]
    assert abs(s.mean() - 1.0 / 3.0) < 1e-12  # magnetisation of the plateau
    rng = np.random.default_rng(3)
    rand = np.where(rng.random((8, L, L)) < 0.5, 1, -1).astype(np.int8)
    assert not learned.plateau_sectors(rand)[2].any()


def test_symmetry_images_change_sector_and_self_maps_do_not():
    s = _ordered()
    base = _sectors(s)
    moved = {
        "two columns": np.roll(s, 2, axis=1),
        "four columns": np.roll(s, 4, axis=1),
        "transpose": s.T.copy(),
        "transpose of two columns": np.roll(s, 2, axis=1).T.copy(),
    }
    same = {
        "itself": s.copy(),
        "three columns": np.roll(s, 3, axis=1),
        "two rows": np.roll(s, 2, axis=0),
        "six columns and four rows": np.roll(np.roll(s, 6, axis=1), 4, axis=0),
    }
    for name, t in moved.items():
        cur = _sectors(t)
        assert cur[2][0], name
        assert learned.sector_changes(base, cur)[0], name
    for name, t in same.items():
        assert not learned.sector_changes(base, _sectors(t))[0], name


def test_thermal_noise_and_disorder_are_not_moves():
    s = _ordered()
    rng = np.random.default_rng(5)
    noisy = s.copy()
    idx = rng.choice(L * L, size=12, replace=False)
    noisy.reshape(-1)[idx] *= -1
    assert not learned.sector_changes(_sectors(s), _sectors(noisy))[0]
    # a disordered state on either side is never counted, whatever its phase
    rand = np.where(rng.random((L, L)) < 0.5, 1, -1).astype(np.int8)
    assert not learned.sector_changes(_sectors(s), _sectors(rand))[0]
    assert not learned.sector_changes(_sectors(rand), _sectors(np.roll(s, 2, axis=1)))[0]
    # per chain: a batch mixes moved and unmoved chains
    prev = _sectors(s, s, s)
    cur = _sectors(s, np.roll(s, 2, axis=1), noisy)
    assert learned.sector_changes(prev, cur).tolist() == [False, True, False]
