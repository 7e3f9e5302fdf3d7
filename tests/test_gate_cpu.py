"""Host logic of the learned start's gate: the relative data jump the step
compares, and the split that minimises Newton iterations (brute force over
every threshold on small seeded cases, ties included)."""
import numpy as np
import pytest

from paper_2602_21911_amd import learn


def test_jump_size_hand_case():
    # left (rho, u, p) = (1, 0, 1), right (2, 0.5, 0.5), gamma 1.4:
    # |dp|/pbar = 0.5/0.75, |drho|/rhobar = 1/1.5, |du|/cbar with
    # c_L = sqrt(1.4), c_R = sqrt(0.35)
    wl = np.array([[1.0, 0.0, 1.0]])
    wr = np.array([[2.0, 0.5, 0.5]])
    cbar = 0.5 * (np.sqrt(1.4) + np.sqrt(0.35))
    want = 0.5 / 0.75 + 1.0 / 1.5 + 0.5 / cbar
    assert learn.jump_size(wl, wr)[0] == pytest.approx(want, rel=1e-15)
    # symmetric in the two sides, zero for equal states
    assert learn.jump_size(wr, wl)[0] == pytest.approx(want, rel=1e-15)
    assert learn.jump_size(wl, wl)[0] == 0.0


def _total(j, a, b, gate):
    # the step's rule: the network above the gate, PVRS at or below it
    return float(np.where(j > gate, b, a).sum())


@pytest.mark.parametrize("seed", range(6))
def test_best_split_is_the_brute_force_minimum(seed):
    rng = np.random.default_rng(seed)
    n = 40
    j = rng.choice(np.linspace(0.0, 3.0, 25), n) if seed % 2 else rng.uniform(0.0, 3.0, n)  # ties on odd seeds
    a = rng.integers(2, 9, n).astype(float)
    b = rng.integers(2, 9, n).astype(float)
    gate, tot, tot_pvrs, tot_learned = learn.best_split(j, a, b)
    assert tot_pvrs == a.sum() and tot_learned == b.sum()
    # every threshold that separates the sorted jumps differently
    cands = np.concatenate([[-1.0], np.unique(j)])
    best = min(_total(j, a, b, g) for g in cands)
    assert tot == best
    assert _total(j, a, b, gate) == best  # the returned gate realises it


def test_best_split_extremes():
    j = np.array([0.5, 1.0, 2.0])
    # the network never helps: every problem stays with PVRS
    gate, tot, _, _ = learn.best_split(j, [3, 3, 3], [5, 5, 5])
    assert gate == 2.0 and tot == 9.0 and _total(j, np.full(3, 3.0), np.full(3, 5.0), gate) == 9.0
    # the network always helps: gate 0 (only identical states keep PVRS)
    gate, tot, _, _ = learn.best_split(j, [5, 5, 5], [3, 3, 3])
    assert gate == 0.0 and tot == 9.0
    # helps above 0.75 only
    gate, tot, _, _ = learn.best_split(j, [3, 5, 6], [4, 4, 4])
    assert gate == 0.75 and tot == 11.0
