"""Pins of the FP64 CPU oracle against facts that do not come from the oracle.

Every check here is independent of the HIP path and of the oracle's own
formulas: textbook constants (NaCl Madelung constant, with Benson's series
re-evaluated here), closed forms (structure factor of a perfect rock-salt
lattice), invariances the exact Ewald sum must satisfy (alpha-independence of
the total energy, translation/permutation/charge-sign symmetry, zero net
force), F = -grad E and dE/dq by central finite differences, brute force on tiny
inputs, and direct spherical-shell image sums (tin-foil limit plus the dipole
term).  The formulas follow section 3 of the paper; see ``oracle/ewald_oracle.c``.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1708_01135_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_value(name):
    with open(os.path.join(GOLDEN, name)) as f:
        vals = [l.strip() for l in f if l.strip() and not l.startswith("#")]
    return float(vals[0])


MADELUNG = _golden_value("madelung_nacl.txt")


def rel(a, b):
    return abs(a - b) / abs(b)


def relF(f, g):
    return np.linalg.norm(f - g) / np.linalg.norm(g)


# ----------------------------------------------------------------- constants

def test_madelung_golden_matches_benson_series():
    m = np.arange(1, 121, 2, dtype=float)
    M2, N2 = np.meshgrid(m, m)
    benson = 12 * np.pi * np.sum(np.cosh(np.pi / 2 * np.sqrt(M2 ** 2 + N2 ** 2)) ** -2)
    assert abs(benson - MADELUNG) < 1e-15


@pytest.mark.parametrize("method", [oracle.BRUTE, oracle.FAST])
def test_madelung_two_site_cube(method):
    # 2x2x2 perfect rock salt, converged (alpha r_c^2 = 36, k_c^2/(4 alpha) = 39)
    pos, q, L = wl.perfect_rock_salt(2)
    en, f, _ = oracle.energy_forces(pos, q, L, 9.1, 1.99, 12, method)
    assert rel(en[0], -len(q) * MADELUNG / 2) < 1e-12
    assert np.abs(f).max() < 1e-12


def test_madelung_8cube_converged():
    pos, q, L = wl.perfect_rock_salt(8)
    en, f, _ = oracle.energy_forces(pos, q, L, 0.9, 7.9, 14, oracle.FAST)
    assert rel(en[0], -256 * MADELUNG) < 1e-12
    assert np.abs(f).max() < 1e-12  # inversion centre on every site


def test_madelung_small_workload_parameters():
    # the 8^3 workload's own (alpha, r_c, K) on the unjittered lattice: only
    # truncation error is left (erfc(sqrt(0.9)*4)/4 ~ 1e-8 per neighbour)
    pos, q, L = wl.perfect_rock_salt(8)
    en, _, _ = oracle.energy_forces(pos, q, L, 0.9, 4.0, 8, oracle.FAST)
    assert rel(en[0], -256 * MADELUNG) < 2e-6


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n_side", [2, 4, 8])
def test_structure_factor_perfect_lattice_closed_form(n_side):
    pos, q, L = wl.perfect_rock_salt(n_side)
    K = min(8, 2 * n_side)
    kv = oracle.kset(K, half=False)
    s = oracle.structure_factor(pos, q, L, kv)
    # S = N where every n_a == n_side/2 (mod n_side), else 0
    special = np.all(np.mod(kv, n_side) == n_side // 2, axis=1)
    expect = np.where(special, float(len(q)), 0.0)
    assert np.abs(s - expect).max() < 1e-12 * len(q)
    # the table route's half-space S_k agrees with the closed form too
    _, _, _, sk = oracle.recip_space(pos, q, L, 1.0, K, oracle.FAST, want_sk=True)
    kh = oracle.kset(K, half=True)
    sp = np.all(np.mod(kh, n_side) == n_side // 2, axis=1)
    assert np.abs(sk - np.where(sp, float(len(q)), 0.0)).max() < 1e-12 * len(q)


def test_kset_counts_by_direct_count():
    for K in (1, 3, 8, 20):
        r = np.arange(-K, K + 1)
        X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
        m2 = X ** 2 + Y ** 2 + Z ** 2
        full = int(np.count_nonzero((m2 > 0) & (m2 <= K * K)))
        assert len(oracle.kset(K, half=False)) == full
        kh = oracle.kset(K, half=True)
        assert 2 * len(kh) == full
        # half space + its negation is the full set, disjoint
        allk = {tuple(v) for v in kh} | {tuple(-v) for v in kh}
        assert len(allk) == full


# --------------------------------------------------------------- invariances

def _jittered(n_side=8, jitter=0.1, seed=3):
    return wl.rock_salt(n_side, jitter, seed)


@pytest.mark.parametrize("neutral", [True, False])
def test_alpha_invariance_converged(neutral):
    pos, q, L = _jittered()
    if not neutral:
        q = q.copy()
        q[:5] += 0.37  # Q != 0: the background term must restore alpha-independence
    energies, parts = [], []
    for alpha in (0.6, 0.9, 1.2):
        K = int(math.ceil(L * math.sqrt(144 * alpha) / (2 * math.pi)))  # k_c^2/(4 alpha) >= 36
        en, _, _ = oracle.energy_forces(pos, q, L, alpha, 7.9, K, oracle.FAST)
        energies.append(en[0])
        parts.append(en[1:])
    for e in energies[1:]:
        assert rel(e, energies[0]) < 1e-10
    # the split itself moves by O(1): the test is not vacuous
    assert abs(parts[0][0] - parts[2][0]) > 1.0


def test_net_force_zero_and_charge_sign_symmetry():
    pos, q, L = _jittered(seed=5)
    for method in (oracle.BRUTE, oracle.FAST):
        en, f, _ = oracle.energy_forces(pos, q, L, 0.9, 4.0, 8, method)
        assert np.abs(f.sum(axis=0)).max() < 1e-12 * np.abs(f).sum()
        en2, f2, _ = oracle.energy_forces(pos, -q, L, 0.9, 4.0, 8, method)
        assert rel(en2[0], en[0]) < 1e-13
        assert relF(f2, f) < 1e-13


def test_translation_and_permutation_invariance():
    pos, q, L = _jittered(seed=7)
    en, f, dq = oracle.energy_forces(pos, q, L, 0.9, 4.0, 8, oracle.FAST)
    shift = np.array([0.37, -5.1, 12.9])
    en2, f2, dq2 = oracle.energy_forces(pos + shift, q, L, 0.9, 4.0, 8, oracle.FAST)
    assert rel(en2[0], en[0]) < 1e-12
    assert relF(f2, f) < 1e-10
    perm = np.random.default_rng(0).permutation(len(q))
    en3, f3, dq3 = oracle.energy_forces(pos[perm], q[perm], L, 0.9, 4.0, 8, oracle.FAST)
    assert rel(en3[0], en[0]) < 1e-13
    assert relF(f3, f[perm]) < 1e-13
    assert np.abs(dq3 - dq[perm]).max() < 1e-12


def test_potential_identity():
    # E = 1/2 sum_i q_i phi_i + E_self + E_bg, phi = dE/dq + 2 sqrt(a/pi) q + pi Q/(V a)
    pos, q = wl.random_neutral(200, 6.0, seed=11, neutral=False)
    L, a = 6.0, 1.3
    en, _, dq = oracle.energy_forces(pos, q, L, a, 2.9, 7, oracle.FAST)
    Q = q.sum()
    phi = dq + 2 * math.sqrt(a / math.pi) * q + math.pi * Q / (L ** 3 * a)
    assert rel(0.5 * np.dot(q, phi) + en[3] + en[4], en[0]) < 1e-12


# ------------------------------------------------------ finite differences

def _energy(pos, q, L, a, rc, K):
    return oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST)[0][0]


@pytest.mark.parametrize("K", [5, 12])
def test_forces_are_minus_energy_gradient(K):
    # converged real space (alpha r_c^2 = 36.5) so no pair crosses the cutoff
    # discontinuity; K=5 leaves the reciprocal sum truncated on purpose
    pos, q, L = wl.rock_salt(4, 0.15, seed=2)
    a, rc = 2.4, 3.9
    _, f, _ = oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST)
    h = 1e-4
    rng = np.random.default_rng(1)
    for i in rng.choice(len(q), 12, replace=False):
        for ax in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, ax] += h
            p2[i, ax] -= h
            fd = -(_energy(p1, q, L, a, rc, K) - _energy(p2, q, L, a, rc, K)) / (2 * h)
            assert abs(fd - f[i, ax]) < 1e-7 * max(1.0, np.sqrt(np.mean(f ** 2)))


def test_dEdq_is_energy_derivative():
    # non-neutral on purpose: the background term contributes -pi Q/(V alpha)
    pos, q = wl.random_neutral(64, 4.0, seed=4, neutral=False)
    assert abs(q.sum()) > 0.5
    L, a, rc, K = 4.0, 2.4, 3.9, 9
    _, _, dq = oracle.energy_forces(pos, q, L, a, rc, K, oracle.FAST)
    h = 1e-4
    for i in (0, 7, 33, 63):
        q1, q2 = q.copy(), q.copy()
        q1[i] += h
        q2[i] -= h
        fd = (_energy(pos, q1, L, a, rc, K) - _energy(pos, q2, L, a, rc, K)) / (2 * h)
        assert abs(fd - dq[i]) < 1e-8 * max(1.0, abs(dq[i]))


# --------------------------------------------------------------- brute force

@pytest.mark.parametrize("case", [
    dict(n=8, L=3.0, a=1.1, rc=2.9, K=5),    # r_c > L/2: several images of one pair
    dict(n=37, L=5.0, a=0.8, rc=2.4, K=6),   # odd count
    dict(n=64, L=4.3, a=1.5, rc=4.3, K=7),   # r_c = L
    dict(n=1, L=2.0, a=2.0, rc=1.9, K=4),    # a single charge (self-images only in k space)
])
def test_cell_list_and_tables_match_brute_force(case):
    pos, q = wl.random_neutral(case["n"], case["L"], seed=case["n"], neutral=case["n"] > 1)
    pos = pos + np.array([-7.0, 3.2, 9.9])  # unwrapped input
    eb, fb, db = oracle.energy_forces(pos, q, case["L"], case["a"], case["rc"], case["K"], oracle.BRUTE)
    ef, ff, df = oracle.energy_forces(pos, q, case["L"], case["a"], case["rc"], case["K"], oracle.FAST)
    for p in range(5):
        assert abs(ef[p] - eb[p]) <= 1e-13 * max(1.0, abs(eb[p]))
    assert np.abs(ff - fb).max() <= 1e-13 * max(1.0, np.abs(fb).max())
    assert np.abs(df - db).max() <= 1e-13 * max(1.0, np.abs(db).max())


def test_real_space_targets_match_full():
    pos, q, L = _jittered(seed=9)
    _, f, ph = oracle.real_space(pos, q, L, 0.9, 4.0, oracle.FAST)
    t = [0, 5, 511, 100]
    _, ft, pt = oracle.real_space(pos, q, L, 0.9, 4.0, oracle.BRUTE, targets=t)
    assert np.abs(ft - f[t]).max() < 1e-13
    assert np.abs(pt - ph[t]).max() < 1e-13


@pytest.mark.parametrize("method", [oracle.BRUTE, oracle.FAST])
def test_target_assembly_matches_full_evaluation(method):
    """The entry point that writes the stored full-size references assembles
    forces and dE/dq of the listed particles; it must reproduce the full
    evaluation (pinned above) at those particles, and its S_k the direct sums."""
    pos, q = wl.random_neutral(300, 7.0, seed=5, neutral=False)
    e, f, d = oracle.energy_forces(pos, q, 7.0, 1.0, 3.4, 9, method)
    t = [3, 17, 299, 0, 150, 17]
    if method == oracle.FAST:
        e2, f2, d2, sk = oracle.energy_forces_targets(pos, q, 7.0, 1.0, 3.4, 9, targets=t, method=method,
                                                      want_sk=True)
        sk_direct = oracle.structure_factor(pos, q, 7.0, oracle.kset(9, half=True))
        assert np.abs(sk - sk_direct).max() < 1e-11
    else:
        e2, f2, d2 = oracle.energy_forces_targets(pos, q, 7.0, 1.0, 3.4, 9, targets=t, method=method)
    assert np.array_equal(e, e2)
    assert np.abs(f2 - f[t]).max() <= 1e-14 * np.abs(f).max()
    assert np.abs(d2 - d[t]).max() <= 1e-14 * np.abs(d).max()
    e3, f3, d3 = oracle.energy_forces_targets(pos, q, 7.0, 1.0, 3.4, 9, method=method)
    assert np.array_equal(f3, f) and np.array_equal(d3, d)


# ----------------------------------------------------- spherical image sums

def _shell_energy(pos, q, L, R):
    """1/2 sum over images n with |n| <= R of sum_{i,j}' q_i q_j / |r_i - r_j + n L|."""
    r = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    sel = X ** 2 + Y ** 2 + Z ** 2 <= R * R
    shifts = L * np.stack([X[sel], Y[sel], Z[sel]], axis=1).astype(float)
    e = 0.0
    n = len(q)
    for i in range(n):
        d = pos[i] - pos  # (n,3)
        dd = d[:, None, :] + shifts[None, :, :]
        r2 = np.einsum("jsk,jsk->js", dd, dd)
        with np.errstate(divide="ignore"):
            inv = 1.0 / np.sqrt(r2)
        inv[~np.isfinite(inv)] = 0.0  # the i == j, n == 0 term
        e += 0.5 * q[i] * np.dot(q, inv.sum(axis=1))
    return e


@pytest.mark.parametrize("seed", [0, 1])
def test_spherical_image_sum_limit_is_tinfoil_plus_dipole(seed):
    rng = np.random.default_rng(seed)
    n, L = 4, 1.7
    pos = rng.uniform(0, L, size=(n, 3))
    q = np.array([1.0, -1.0, 0.5, -0.5])
    en, _, _ = oracle.energy_forces(pos, q, L, 9.0, 1.69, 14, oracle.FAST)  # converged
    M = q @ pos
    target = en[0] + 2 * math.pi * (M @ M) / (3 * L ** 3)
    # shell sums converge like 1/R^2; Richardson-extrapolate two radii
    r1, r2 = 24, 34
    e1, e2 = _shell_energy(pos, q, L, r1), _shell_energy(pos, q, L, r2)
    extrap = (e2 * r2 ** 2 - e1 * r1 ** 2) / (r2 ** 2 - r1 ** 2)
    assert abs(extrap - target) < 5e-6 * abs(target)
    # the dipole term matters at this size: tin-foil alone is clearly off
    assert abs(e2 - en[0]) > 10 * abs(extrap - target)
