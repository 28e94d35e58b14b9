"""Pins for the FP64 CPU oracle (no GPU).

Each test checks the oracle against something other than itself: the
brute-force form of Eq. 2 written independently in numpy, conservation laws,
detailed balance, closed forms from Fermi's golden rule, finite differences
(exact up to rounding because I is quadratic in f and linear in |g|^2),
the RK4 amplification polynomial and the Drude mobility.
"""
import math

import numpy as np
import pytest

import oracle
import synth

HBAR = 0.6582119569          # eV fs
KB = 8.617333262e-5          # eV/K


@pytest.fixture(scope="module")
def c1():
    s = synth.parabolic_system(8)
    return s, synth.c1_occupations(s), s.nph(300.0)


def _G(x, sig):
    return math.exp(-0.5 * (x / sig) ** 2) / (sig * math.sqrt(2 * math.pi))


# --------------------------------------------------------------- brute force
@pytest.mark.parametrize("maker", [lambda: synth.parabolic_system(4),
                                   lambda: synth.multiband_system(),
                                   lambda: synth.multiband_system(kn=4, qn=2, nb=3, n_k=10, seed=5)])
def test_list_equals_brute_force_tiny(maker):
    """Channel-list loop == Eq. 2 summed over the full q grid, bands and modes
    (Eq. 2; pairing of the two contributions of a channel: GPU algorithm step 1)."""
    s = maker()
    f = synth.random_occupations(s, 5)
    nph = s.nph(300.0)
    I = oracle.collision(s, f, nph)
    Ib = oracle.collision_brute(s, f, nph)
    assert np.abs(I - Ib).max() <= 1e-14 * np.abs(Ib).max()


def test_c1_counts_and_brute_force(c1):
    s, f, nph = c1
    assert s.n_states == 512
    assert s.n_channels == 512 * 511 // 2 * 3
    I = oracle.collision(s, f, nph)
    Ib = oracle.collision_brute(s, f, nph)
    assert np.abs(I - Ib).max() <= 1e-14 * np.abs(Ib).max()


# --------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_particle_number_conserved(seed):
    """sum_s I_s = 0 for any f: each channel moves an electron between two states."""
    s = synth.multiband_system(seed=seed + 20)
    f = synth.random_occupations(s, seed)
    I = oracle.collision(s, f, s.nph(250.0))
    gross = np.abs(I).sum()
    assert abs(I.sum()) <= 1e-14 * gross


def test_pauli_blocking(c1):
    """Empty and completely full bands do not scatter."""
    s, _, nph = c1
    assert np.all(oracle.collision(s, np.zeros(s.n_states), nph) == 0.0)
    assert np.all(oracle.collision(s, np.ones(s.n_states), nph) == 0.0)


def test_in_minus_out_is_the_collision_integral(c1):
    """Gross in- and out-scattering rates recombine to I (same Eq. 2 terms
    regrouped by occupation product), and both are non-negative."""
    s, f, nph = c1
    rin, rout = oracle.collision_inout(s, f, nph)
    I = oracle.collision(s, f, nph)
    assert np.all(rin >= 0) and np.all(rout >= 0)
    assert np.abs((rin - rout) - I).max() <= 1e-14 * rout.max()


def test_linear_in_g2(c1):
    s, f, nph = c1
    I1 = oracle.collision(s, f, nph)
    I3 = oracle.collision(s, f, nph, g2=3.0 * s.g2)
    assert np.allclose(I3, 3.0 * I1, rtol=1e-14, atol=0)


def test_detailed_balance_resonant_ladder():
    """Fermi-Dirac electrons with Bose-Einstein phonons at the same T are a
    fixed point when every channel is on resonance (counter-process Gaussian
    underflows): I = 0 to rounding.  With electrons hotter than the phonons
    the same system relaxes (I != 0)."""
    s = synth.ladder_system()
    nph = s.nph(300.0)
    f_eq = synth.fermi_dirac(s.eps, 0.1, 300.0)
    I_eq = oracle.collision(s, f_eq, nph)
    f_hot = synth.fermi_dirac(s.eps, 0.1, 900.0)
    I_hot = oracle.collision(s, f_hot, nph)
    assert np.abs(I_hot).max() > 0
    assert np.abs(I_eq).max() <= 1e-13 * np.abs(I_hot).max()


def test_two_state_golden_rule():
    """One channel, the upper state exactly one phonon above the lower one.
    Golden rule: the lower state gains (N+1) f2 (1-f1) by emission from the
    upper one and loses N f1 (1-f2) by absorption, at rate
    (2 pi / hbar) |g|^2 / N_q * G(0); the upper state loses the same amount."""
    s = synth.two_state_system(dE=0.05, hw=0.05, g2=2e-3, sigma=0.004, nq=2)
    T = 300.0
    N = 1.0 / math.expm1(0.05 / (KB * T))
    nph = np.full((2, 1), N)
    f = np.array([0.7, 0.2])
    I = oracle.collision(s, f, nph)
    rate = 2 * math.pi / HBAR * 2e-3 / 2 * _G(0.0, 0.004)
    expect1 = rate * ((N + 1) * f[1] * (1 - f[0]) - N * f[0] * (1 - f[1]))
    assert I[0] == pytest.approx(expect1, rel=1e-13)
    assert I[1] == pytest.approx(-expect1, rel=1e-13)


def test_two_state_off_resonance_tail():
    """Detuned pair: absorption and emission Gaussians are evaluated at
    e1 - e2 + hw and e1 - e2 - hw respectively."""
    sig = 0.01
    s = synth.two_state_system(dE=0.03, hw=0.05, g2=1e-3, sigma=sig, nq=1)
    N = 0.4
    nph = np.full((1, 1), N)
    f = np.array([0.3, 0.6])
    I = oracle.collision(s, f, nph)
    pref = 2 * math.pi / HBAR * 1e-3
    de = -0.03
    absorb = _G(de + 0.05, sig) * (N * f[0] * (1 - f[1]) - (N + 1) * f[1] * (1 - f[0]))
    emit = _G(de - 0.05, sig) * ((N + 1) * f[0] * (1 - f[1]) - N * f[1] * (1 - f[0]))
    assert I[0] == pytest.approx(-pref * (absorb + emit), rel=1e-13)


# --------------------------------------------------------- channel selection
@pytest.mark.parametrize("swap", [False, True])
def test_selection_two_state_by_hand(swap):
    """One channel, e_j - e_i = 0.07 eV.  With hw = 0.03 eV the emission
    Gaussian sits 0.04 eV = 5 sigma from its centre and the absorption one
    0.10 eV; with hw = 0.2 eV the nearest is absorption at 0.13 eV = 16.25
    sigma.  The channel survives exactly when n_sigma exceeds that distance,
    in either orientation; the |g|^2 cut keeps |g|^2 >= g2_min."""
    def mk(hw):
        s = synth.two_state_system(dE=0.07, hw=hw, g2=2e-3, sigma=0.008, nq=2)
        if swap:
            s.ch_i, s.ch_j = s.ch_j.copy(), s.ch_i.copy()
        return s
    s = mk(0.03)
    assert not oracle.select_channels(s, 4.9)[0]
    assert oracle.select_channels(s, 5.1)[0]
    s = mk(0.2)
    assert not oracle.select_channels(s, 16.2)[0]
    assert oracle.select_channels(s, 16.3)[0]
    assert oracle.select_channels(s, 0.0, 2e-3)[0]
    assert not oracle.select_channels(s, 0.0, 2.0001e-3)[0]
    assert not oracle.select_channels(s, 16.3, 2.0001e-3)[0]


def test_selection_disabled_keeps_everything(c1):
    s, _, _ = c1
    assert oracle.select_channels(s).all()
    assert oracle.select_channels(s, 1e4, 0.0).all()
    assert oracle.channel_phonon_energy(s).min() > 0


@pytest.mark.parametrize("nsig,g2min", [(2.0, 0.0), (3.0, 5e-4), (0.0, 2e-3)])
def test_selection_changes_I_by_at_most_the_dropped_tails(c1, nsig, g2min):
    """A dropped channel contributes |X| <= C |g|^2 (N+1) (G(Delta+hw) +
    G(Delta-hw)) to each of its two states (Eq. 2 with 0 <= f <= 1).  Energy-cut
    channels have both Gaussians below G(n sigma), |g|^2-cut ones below G(0);
    so I(all) - I(kept) is bounded state by state.  A selection that dropped a
    near-resonant channel it should keep would break the bound."""
    s, f, nph = c1
    keep = oracle.select_channels(s, nsig, g2min)
    assert 0 < keep.sum() < keep.size
    diff = oracle.collision(s, f, nph) - oracle.collision(oracle.subset(s, keep), f, nph)
    w = oracle.channel_phonon_energy(s)
    N = 1.0 / np.expm1(w / (KB * 300.0))
    C = 2 * math.pi / (HBAR * s.n_q_norm)
    sig = s.sigma
    g0 = 1.0 / (sig * math.sqrt(2 * math.pi))
    e_cut = ~oracle.select_channels(s, nsig)
    gmax = np.where(e_cut, math.exp(-0.5 * nsig ** 2) * g0, g0)
    per = np.where(keep, 0.0, C * s.g2 * (N + 1) * 2 * gmax)
    bound = np.zeros(s.n_states)
    np.add.at(bound, s.ch_i, per)
    np.add.at(bound, s.ch_j, per)
    assert np.all(np.abs(diff) <= bound * (1 + 1e-12) + 1e-300)
    assert np.abs(diff).max() > 0


# ------------------------------------------------------- elastic mechanism
def test_elastic_two_state_by_hand():
    """One defect channel between states 10 meV apart: I_1 = C |g|^2 G(-0.01)
    (f_2 - f_1), I_2 = -I_1, with C = 2 pi / (hbar N_q); Eq. 2 at hw = 0 and
    N = 0 gives the same numbers."""
    sig, g2, nq = 0.008, 3e-3, 2
    s = synth.two_state_system(dE=0.01, hw=0.0, g2=g2, sigma=sig, nq=nq)
    f = np.array([0.8, 0.3])
    C = 2 * math.pi / (HBAR * nq)
    expect = C * g2 * _G(-0.01, sig) * (0.3 - 0.8)
    I = oracle.collision_elastic(s, f)
    assert I[0] == pytest.approx(expect, rel=1e-14)
    assert I[1] == pytest.approx(-expect, rel=1e-14)
    I2 = oracle.collision(s, f, np.zeros((nq, 1)))
    assert np.allclose(I2, I, rtol=1e-14, atol=0)


def test_elastic_is_eq2_without_phonons():
    """On every channel of a defect system, Eq. 2 (the C loop) with hw = 0 and
    N = 0 equals the numpy elastic form, and the phonon channels beside it add
    on top."""
    s = synth.defect_system(4, with_phonons=True)
    f = synth.random_occupations(s, 12)
    nph = s.nph(300.0)
    e = s.meta["elastic_mode"]
    I_el = oracle.collision_elastic(s, f, modes=[e])
    sub = oracle.subset(s, np.asarray(s.ch_nu) == e)
    I_eq2 = oracle.collision(sub, f, nph)
    assert np.abs(I_eq2 - I_el).max() <= 1e-14 * np.abs(I_el).max()
    ph = oracle.subset(s, np.asarray(s.ch_nu) != e)
    I_all = oracle.collision(s, f, nph)
    assert np.abs(I_all - (I_el + oracle.collision(ph, f, nph))).max() <= 1e-13 * np.abs(I_all).max()


def test_elastic_dissipation_identity():
    """The elastic operator is symmetric and dissipative: sum_d f_d I_d =
    -sum_c C |g|^2 G (f_i - f_j)^2 <= 0; constants are its null space and
    particle number is conserved."""
    s = synth.defect_system(4, with_phonons=False)
    f = synth.random_occupations(s, 3)
    I = oracle.collision_elastic(s, f)
    i, j = s.ch_i, s.ch_j
    d = s.eps[i] - s.eps[j]
    G = np.exp(-0.5 * (d / s.sigma) ** 2) / (s.sigma * math.sqrt(2 * math.pi))
    C = 2 * math.pi / (HBAR * s.n_q_norm)
    q = -np.sum(C * s.g2 * G * (f[i] - f[j]) ** 2)
    assert q < 0
    assert float(f @ I) == pytest.approx(q, rel=1e-12)
    assert abs(I.sum()) <= 1e-13 * np.abs(I).max()
    assert np.abs(oracle.collision_elastic(s, np.full(s.n_states, 0.37))).max() == 0.0


# ------------------------------------------------- phonon side (dN/dt)
def _fine_ladder():
    """The resonant ladder with every k doubled on a k grid twice as fine
    as the q grid: pairs stay commensurate and N_k = 8 N_q."""
    import copy
    s = synth.ladder_system()
    r = copy.copy(s)
    kg = np.asarray(s.kgrid)
    c = synth.grid_coords(s.kgrid)[s.state_k] * 2
    r.kgrid = tuple(int(x) for x in 2 * kg)
    r.state_k = synth.linear_index(c, r.kgrid).astype(np.int32)
    return r


def test_phonon_rate_two_state_by_hand():
    """One channel on a 3-point ring: q = 1 and -q = 2 get the emission minus
    absorption of their own processes, q = 0 gets nothing."""
    dE, hw, g2, sig, N = 0.045, 0.05, 2e-3, 0.01, 0.3
    s = synth.two_state_system(dE=dE, hw=hw, g2=g2, sigma=sig, nq=3)
    f = np.array([0.2, 0.7])
    nph = np.full((3, 1), N)
    dN = oracle.phonon_rate(s, f, nph)[:, 0]
    Cp = 2 * math.pi / (HBAR * 3)
    up = Cp * g2 * _G(-dE + hw, sig) * ((N + 1) * f[1] * (1 - f[0]) - N * f[0] * (1 - f[1]))
    dn = Cp * g2 * _G(-dE - hw, sig) * ((N + 1) * f[0] * (1 - f[1]) - N * f[1] * (1 - f[0]))
    assert dN[0] == 0.0
    assert dN[1] == pytest.approx(up, rel=1e-14)
    assert dN[2] == pytest.approx(dn, rel=1e-14)


def test_phonon_rate_conserves_energy_with_the_electrons():
    """On a resonant system every process moves exactly hw between the
    electrons and one phonon: (1/N_k) sum e_s I_s + (1/N_q) sum hw dN = 0,
    with I from the C loop of Eq. 2 (N_k = 8 N_q here)."""
    s = _fine_ladder()
    assert np.prod(s.kgrid) == 8 * np.prod(s.qgrid)
    f = 0.3 + 0.4 * synth.random_occupations(s, 5)
    nph = np.full_like(s.hw, 0.7)
    I = oracle.collision(s, f, nph)
    dN = oracle.phonon_rate(s, f, nph)
    e_el = float(s.eps @ I) / np.prod(s.kgrid)
    e_ph = float((s.hw * dN).sum()) / np.prod(s.qgrid)
    assert abs(e_ph) > 0
    assert abs(e_el + e_ph) <= 1e-13 * abs(e_ph)


def test_phonon_rate_detailed_balance_and_empty_bands():
    """At Fermi-Dirac / Bose-Einstein equilibrium of one temperature the
    resonant processes balance, so dN = 0; empty and full bands give 0."""
    s = _fine_ladder()
    T = 300.0
    f = synth.fermi_dirac(s.eps, 0.1, T)
    nph = s.nph(T)
    hot = oracle.phonon_rate(s, synth.fermi_dirac(s.eps, 0.1, 2 * T), nph)
    assert np.abs(hot).max() > 0
    assert np.abs(oracle.phonon_rate(s, f, nph)).max() <= 1e-13 * np.abs(hot).max()
    assert np.abs(oracle.phonon_rate(s, np.zeros(s.n_states), nph)).max() == 0.0
    assert np.abs(oracle.phonon_rate(s, np.ones(s.n_states), nph)).max() == 0.0


def test_coupled_rk4_keeps_energy_and_particles():
    """Electrons and phonons stepped together: total energy per cell
    (1/N_k) sum e f + (1/N_q) sum hw N and the electron count are linear
    invariants of the resonant system, which RK4 keeps to rounding, while the
    phonons do change; at a common-temperature equilibrium nothing moves."""
    s = _fine_ladder()
    nk, nq = float(np.prod(s.kgrid)), float(np.prod(s.qgrid))
    f = 0.2 + 0.5 * synth.random_occupations(s, 8)
    N = np.full_like(s.hw, 0.4)
    etot = lambda f_, N_: float(s.eps @ f_) / nk + float((s.hw * N_).sum()) / nq
    e0, n0 = etot(f, N), f.sum()
    f1, N1 = f, N
    for _ in range(5):
        f1, N1 = oracle.rk4_coupled_step(s, f1, N1, 0.5)
    assert np.abs(N1 - N).max() > 1e-6
    assert abs(etot(f1, N1) - e0) <= 1e-13 * abs(e0)
    assert abs(f1.sum() - n0) <= 1e-13 * n0
    T = 300.0
    feq, Neq = synth.fermi_dirac(s.eps, 0.1, T), s.nph(T)
    f2, N2 = oracle.rk4_coupled_step(s, feq, Neq, 0.5)
    assert np.abs(f2 - feq).max() <= 1e-13 and np.abs(N2 - Neq).max() <= 1e-13 * Neq.max()


def test_coupled_rk4_fourth_order():
    """The error of one coupled step against a fine-step solution, over the
    same interval, is 16 times that of two half steps for a fourth-order
    method (2^5 / 2), electrons and phonons alike; a stage input left at the
    step's start drops it towards 4."""
    s = synth.multiband_system()
    f0 = 0.1 + 0.8 * synth.random_occupations(s, 3)
    N0 = s.nph(300.0) * 1.5

    def run(dt, n):
        f, N = f0, N0
        for _ in range(n):
            f, N = oracle.rk4_coupled_step(s, f, N, dt)
        return f, N
    T = 0.5
    fr, Nr = run(T / 64, 64)
    f1, N1 = run(T, 1)
    f2, N2 = run(T / 2, 2)
    rf = np.abs(f1 - fr).max() / np.abs(f2 - fr).max()
    rN = np.abs(N1 - Nr).max() / np.abs(N2 - Nr).max()
    assert np.abs(N1 - N0).max() > 1e-6
    assert 12 < rf < 24 and 12 < rN < 24, (rf, rN)


# ------------------------------------------------------ drift term (Eq. 1)
def _ring(n=16, with_channels=False):
    """One band on an n x 1 x 1 periodic grid, every state present."""
    s = synth.parabolic_system(4)
    import copy
    r = copy.copy(s)
    r.kgrid = r.qgrid = (n, 1, 1)
    r.state_k = np.arange(n, dtype=np.int32)
    r.state_band = np.zeros(n, np.int8)
    r.eps = 0.01 * np.arange(n, dtype=np.float64)
    r.hw = np.full((n, 1), 0.03)
    r.n_modes = 1
    r.ch_i = np.zeros(0, np.int32)
    r.ch_j = np.zeros(0, np.int32)
    r.ch_nu = np.zeros(0, np.int8)
    r.g2 = np.zeros(0)
    r.n_q_norm = float(n)
    return r


def test_drift_plane_wave_closed_form():
    """On a full periodic grid cos(theta c_x) is an eigenvector pair of the
    central difference: D = r_x sin(theta) sin(theta c_x) for each state."""
    s = synth.parabolic_system(8)
    c = synth.grid_coords(s.kgrid)[s.state_k]
    th = 2 * math.pi * 3 / 8
    f = np.cos(th * c[:, 0])
    r = np.array([0.21, -0.4, 0.05])
    D = oracle.drift(s, f, r)
    assert np.allclose(D, r[0] * math.sin(th) * np.sin(th * c[:, 0]), rtol=0, atol=1e-15)
    g = 0.3 + 0.2 * np.cos(2 * math.pi * c[:, 1] / 8) - 0.1 * np.sin(2 * math.pi * 2 * c[:, 2] / 8)
    Dg = oracle.drift(s, g, r)
    ty, tz = 2 * math.pi / 8, 2 * math.pi * 2 / 8
    expect = (r[1] * 0.2 * math.sin(ty) * np.sin(ty * c[:, 1])
              + r[2] * 0.1 * math.sin(tz) * np.cos(tz * c[:, 2]))
    assert np.allclose(Dg, expect, rtol=0, atol=1e-15)


def test_drift_window_edge_and_transpose():
    """A neighbour outside the window counts as f = 0; with the neighbour
    relation symmetric the operator is antisymmetric (D^T = -D), and on the
    full periodic grid it conserves particle number."""
    s = synth.multiband_system()
    f = synth.random_occupations(s, 2)
    lam = np.random.default_rng(1).normal(size=s.n_states)
    r = np.array([0.3, -0.2, 0.1])
    nbr = oracle.drift_neighbors(s)
    assert (nbr < 0).any() and (nbr >= 0).any()
    D = oracle.drift(s, f, r, nbr)
    # the same states inside a full grid (every k of every band), the added
    # states empty: no neighbour is missing there, and D must not change
    import copy
    nb = int(s.state_band.max()) + 1
    nk = int(np.prod(s.kgrid))
    full = copy.copy(s)
    full.state_k = np.repeat(np.arange(nk, dtype=np.int32), nb)
    full.state_band = np.tile(np.arange(nb, dtype=np.int8), nk)
    pos = {(int(k), int(b)): i for i, (k, b) in enumerate(zip(full.state_k, full.state_band))}
    idx = np.array([pos[(int(k), int(b))] for k, b in zip(s.state_k, s.state_band)])
    ff = np.zeros(nk * nb)
    ff[idx] = f
    assert (oracle.drift_neighbors(full) >= 0).all()
    assert np.allclose(oracle.drift(full, ff, r)[idx], D, rtol=0, atol=1e-15)
    assert np.allclose(oracle.drift_transpose(s, lam, r, nbr), -oracle.drift(s, lam, r, nbr),
                       rtol=0, atol=1e-15)
    assert float(lam @ D) == pytest.approx(float(oracle.drift_transpose(s, lam, r, nbr) @ f), rel=1e-12)
    full = synth.parabolic_system(6)
    Df = oracle.drift(full, synth.random_occupations(full, 4), r)
    assert abs(Df.sum()) <= 1e-14 * np.abs(Df).max()


def test_rk4_pure_drift_amplification():
    """No channels, a periodic ring: a plane wave e^{i theta c} has drift
    eigenvalue -i r sin(theta), so one RK4 step multiplies it by the stability
    polynomial of z = -i r sin(theta) dt."""
    n, r, dt = 16, 0.35, 0.8
    s = _ring(n)
    c = np.arange(n)
    th = 2 * math.pi * 5 / n
    z = -1j * r * math.sin(th) * dt
    P = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    f = np.cos(th * c)
    out = oracle.rk4_step(s, f, np.zeros((n, 1)), dt, rates=[r, 0.0, 0.0])
    assert np.allclose(out, (P * np.exp(1j * th * c)).real, rtol=0, atol=1e-15)


def test_rk4_adjoint_with_drift_matches_finite_differences():
    """Discrete adjoint through RK4 steps with collisions and drift: dL/df0
    and dL/d|g|^2 against central differences (L linear in f_T, the map
    quadratic per stage: differences with a small step are accurate to 1e-7)."""
    s = synth.multiband_system()
    f0 = synth.random_occupations(s, 6) * 0.5
    nph = s.nph(300.0)
    r = np.array([0.02, -0.015, 0.01])
    gT = np.random.default_rng(3).normal(size=s.n_states)
    dt, n = 2.0, 3
    fT, gf, gg = oracle.rk4_trajectory_grad(s, f0, nph, dt, n, gT, rates=r)
    L = lambda ff, g2=None: float(gT @ _roll(s, ff, nph, dt, n, r, g2))
    v = np.random.default_rng(4).normal(size=s.n_states)
    h = 1e-4
    fd = (L(f0 + h * v) - L(f0 - h * v)) / (2 * h)
    assert fd == pytest.approx(float(gf @ v), rel=1e-7)
    w = np.random.default_rng(5).normal(size=s.n_channels) * s.g2
    fd2 = (L(f0, s.g2 + h * w) - L(f0, s.g2 - h * w)) / (2 * h)
    assert fd2 == pytest.approx(float(gg @ w), rel=1e-7)


def _roll(s, f, nph, dt, n, r, g2):
    for _ in range(n):
        f = oracle.rk4_step(s, f, nph, dt, g2=g2, rates=r)
    return f


# --------------------------------------------------------------- derivatives
def test_vjp_matches_central_differences():
    """I is quadratic in f and linear in |g|^2, so central differences are exact
    up to rounding; the hand-written reverse mode must reproduce them."""
    s = synth.multiband_system()
    f = synth.random_occupations(s, 8)
    nph = s.nph(300.0)
    lam = np.random.default_rng(4).normal(size=s.n_states)
    gf, gg = oracle.collision_vjp(s, f, nph, lam)
    h = 1e-3
    fd_f = np.empty(s.n_states)
    for k in range(s.n_states):
        e = np.zeros(s.n_states)
        e[k] = h
        fd_f[k] = lam @ (oracle.collision(s, f + e, nph) - oracle.collision(s, f - e, nph)) / (2 * h)
    assert np.abs(gf - fd_f).max() <= 1e-10 * np.abs(fd_f).max()
    fd_g = np.empty(s.n_channels)
    for c in range(s.n_channels):
        g2 = s.g2.copy()
        g2[c] += s.g2[c]
        fd_g[c] = lam @ (oracle.collision(s, f, nph, g2=g2) - oracle.collision(s, f, nph)) / s.g2[c]
    assert np.abs(gg - fd_g).max() <= 1e-10 * np.abs(fd_g).max()


def test_vjp_euler_identity(c1):
    """L = lam . I is homogeneous of degree 1 in |g|^2: sum_c g2_c dL/dg2_c = L."""
    s, f, nph = c1
    lam = np.random.default_rng(1).normal(size=s.n_states)
    _, gg = oracle.collision_vjp(s, f, nph, lam)
    L = lam @ oracle.collision(s, f, nph)
    assert (s.g2 @ gg) == pytest.approx(L, rel=1e-12)


# --------------------------------------------------------------- RK4
def test_rk4_degenerate_pair_amplification():
    """Two degenerate states (e1 = e2): absorption and emission weights are
    equal, the equation is linear, d(f1-f2)/dt = -2a (f1-f2) with
    a = (2 pi/hbar)(|g|^2/N_q) G(hw) (2N+1), and one RK4 step multiplies
    f1 - f2 by 1 - z + z^2/2 - z^3/6 + z^4/24, z = 2 a dt."""
    sig, hw, g2, N = 0.02, 0.01, 1e-3, 0.7
    s = synth.two_state_system(dE=0.0, hw=hw, g2=g2, sigma=sig, nq=1)
    nph = np.full((1, 1), N)
    a = 2 * math.pi / HBAR * g2 * _G(hw, sig) * (2 * N + 1)
    dt = 0.2
    z = 2 * a * dt
    R = 1 - z + z * z / 2 - z ** 3 / 6 + z ** 4 / 24
    f = np.array([0.9, 0.1])
    d0 = f[0] - f[1]
    for n in range(1, 6):
        f = oracle.rk4_step(s, f, nph, dt)
        assert (f[0] - f[1]) == pytest.approx(d0 * R ** n, rel=1e-12)
        assert f.sum() == pytest.approx(1.0, rel=1e-15)


def test_rk4_fourth_order():
    s = synth.multiband_system()
    f0 = synth.random_occupations(s, 2)
    nph = s.nph(300.0)
    def run(dt, n):
        f = f0.copy()
        for _ in range(n):
            f = oracle.rk4_step(s, f, nph, dt)
        return f
    ref = run(0.25, 64)
    e1 = np.abs(run(2.0, 8) - ref).max()
    e2 = np.abs(run(1.0, 16) - ref).max()
    assert 12.0 < e1 / e2 < 20.0


def _mean_energy(s, f):
    return (s.eps @ f) / f.sum()


def test_rk4_adjoint_matches_finite_differences():
    """Discrete RK4 adjoint of L = sum eps f_T / sum f_T through 4 steps."""
    s = synth.multiband_system(n_k=10, seed=23)
    f0 = synth.random_occupations(s, 9) * 0.8 + 0.1
    nph = s.nph(300.0)
    dt, n = 0.5, 4
    fT = f0.copy()
    for _ in range(n):
        fT = oracle.rk4_step(s, fT, nph, dt)
    gT = (s.eps * fT.sum() - s.eps @ fT) / fT.sum() ** 2
    _, gf0, gg2 = oracle.rk4_trajectory_grad(s, f0, nph, dt, n, gT)
    def L(f0_, g2_=None):
        f = f0_.copy()
        for _ in range(n):
            f = oracle.rk4_step(s, f, nph, dt, g2=g2_)
        return _mean_energy(s, f)
    h = 1e-5
    for k in range(0, s.n_states, 3):
        e = np.zeros(s.n_states)
        e[k] = h
        fd = (L(f0 + e) - L(f0 - e)) / (2 * h)
        assert gf0[k] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(gf0).max())
    for c in range(0, s.n_channels, 7):
        g = s.g2.copy()
        hc = 1e-4 * g[c]
        gp, gm = g.copy(), g.copy()
        gp[c] += hc
        gm[c] -= hc
        fd = (L(f0, gp) - L(f0, gm)) / (2 * hc)
        assert gg2[c] == pytest.approx(fd, rel=1e-5, abs=1e-8 * np.abs(gg2).max())


# --------------------------------------------------------------- transport
def test_transport_coeffs_are_the_jacobian():
    """tau_inv and W are dI/df at f0 (diagonal and off-diagonal)."""
    s = synth.multiband_system()
    f0 = synth.fermi_dirac(s.eps, 0.05, 300.0)
    nph = s.nph(300.0)
    tau_inv, Wij, Wji = oracle.transport_coeffs(s, f0, nph)
    S = s.n_states
    J = np.zeros((S, S))
    h = 1e-3
    for k in range(S):
        e = np.zeros(S)
        e[k] = h
        J[:, k] = (oracle.collision(s, f0 + e, nph) - oracle.collision(s, f0 - e, nph)) / (2 * h)
    Jw = np.zeros((S, S))
    np.add.at(Jw, (s.ch_i, s.ch_j), Wij)
    np.add.at(Jw, (s.ch_j, s.ch_i), Wji)
    Jw[np.diag_indices(S)] -= tau_inv
    assert np.abs(J - Jw).max() <= 1e-10 * np.abs(J).max()


def test_drude_mobility_rta():
    """Constant relaxation time, parabolic band, non-degenerate statistics:
    mu = e tau / m*, here evaluated in SI units independently of the oracle."""
    m_eff, tau_fs, T = 0.3, 25.0, 300.0
    eps, vel = synth.parabolic_states(n=60, a=20.0, m_eff=m_eff)
    f0 = synth.fermi_dirac(eps, -0.2, T)
    x = tau_fs * vel * oracle.dfde_fd(f0, T)[:, None]
    mu = oracle.mobility_cm2(vel, x, f0)
    e_si, me_si = 1.602176634e-19, 9.1093837015e-31
    drude = e_si * tau_fs * 1e-15 / (m_eff * me_si) * 1e4
    assert mu[0, 0] == pytest.approx(drude, rel=2e-4)
    assert mu[1, 1] == pytest.approx(mu[0, 0], rel=1e-12)
    assert abs(mu[0, 1]) < 1e-9 * mu[0, 0]


def test_transport_fixed_point_equals_direct_solve():
    """The iteration x <- tau (v df0/de + W x) started from the RTA solution
    converges to the solution of the linear system (1/tau - W) x = v df0/de,
    obtained here by a dense least-squares solve."""
    s = synth.tb_system(kn=20, qn=10, target_states=300, sigma=0.05)
    T = 300.0
    f0 = synth.fermi_dirac(s.eps, -0.1, T)
    nph = s.nph(T)
    out = oracle.transport_solve(s, f0, s.vel, T, nph, tol=1e-12, max_iter=500)
    assert out["converged"]
    tau_inv, Wij, Wji = oracle.transport_coeffs(s, f0, nph)
    S = s.n_states
    W = np.zeros((S, S))
    np.add.at(W, (s.ch_i, s.ch_j), Wij)
    np.add.at(W, (s.ch_j, s.ch_i), Wji)
    b = s.vel * oracle.dfde_fd(f0, T)[:, None]
    x_direct = np.linalg.lstsq(np.diag(tau_inv) - W, b, rcond=None)[0]
    mu_direct = oracle.mobility_cm2(s.vel, x_direct, f0)
    assert np.abs(out["mu"] - mu_direct).max() <= 1e-9 * np.abs(mu_direct).max()
    x = out["x"]
    resid = x - (b + oracle.transport_apply_W(s, Wij, Wji, x)) / tau_inv[:, None]
    assert np.abs(resid).max() <= 1e-9 * np.abs(x).max()
    assert np.all(np.diag(out["mu"]) > 0)


def test_transport_stops_at_precision_floor():
    """With a tolerance below what FP64 can resolve, the iteration stops once
    the relative mobility change has not set a new minimum for 5 iterations,
    at a change near the rounding level, before max_iter."""
    s = synth.tb_system(kn=20, qn=10, target_states=300, sigma=0.05)
    T = 300.0
    f0 = synth.fermi_dirac(s.eps, -0.1, T)
    out = oracle.transport_solve(s, f0, s.vel, T, s.nph(T), tol=0.0, max_iter=3000)
    assert out["stagnated"] and not out["converged"]
    assert out["iters"] < 3000
    assert out["resid"] < 1e-13
    hist = np.array([np.abs(h).max() for h in out["history"]])
    assert np.all(np.isfinite(hist))


def test_c1_matches_stored_oracle_sample(c1):
    """Regression fixture written by tests/golden/make_golden.py (oracle only)."""
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle_sample.json")) as fh:
        g = json.load(fh)
    s, f, nph = c1
    I = oracle.collision(s, f, nph)
    assert s.n_channels == g["n_channels"]
    assert np.allclose(I[g["states"]], g["I"], rtol=1e-13, atol=1e-13 * g["max_abs"])


def test_collision_threads_is_the_channel_loop():
    """The threaded oracle runs the same C loop over slices of the list: with
    one thread it is bitwise the sequential loop, with several it differs only
    by the order of the additions."""
    for s in (synth.multiband_system(), synth.random_channel_system(n_states=60, n_channels=900, seed=3)):
        f = synth.random_occupations(s, 8)
        nph = s.nph(300.0)
        ref = oracle.collision(s, f, nph)
        assert np.array_equal(oracle.collision_threads(s, f, nph, threads=1), ref)
        for t in (2, 5, 16):
            got = oracle.collision_threads(s, f, nph, threads=t)
            assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_collision_inout_threads_is_the_channel_loop():
    s = synth.multiband_system()
    f = synth.random_occupations(s, 9)
    nph = s.nph(300.0)
    rin, rout = oracle.collision_inout(s, f, nph)
    tin, tout = oracle.collision_inout_threads(s, f, nph, threads=1)
    assert np.array_equal(tin, rin) and np.array_equal(tout, rout)
    tin, tout = oracle.collision_inout_threads(s, f, nph, threads=6)
    assert np.abs(tin - rin).max() <= 1e-14 * rin.max() and np.abs(tout - rout).max() <= 1e-14 * rout.max()


# ------------------------------------------------ reverse mode in N and of the phonon side
def _uneven_bath(s, seed):
    """A positive phonon table that is NOT even in q, so that a q / -q mix-up
    in a reverse mode changes the result."""
    rng = np.random.default_rng(seed)
    return s.nph(300.0) * rng.uniform(0.5, 1.5, size=s.hw.shape)


@pytest.mark.parametrize("maker", [synth.multiband_system, lambda: synth.parabolic_system(4)])
def test_collision_vjp_nph_finite_differences_and_euler(maker):
    """I is affine in N (Eq. 2 with the golden-rule factors), so central
    differences of lam . I along any direction of N are exact up to rounding,
    and sum_q N dL/dN = lam . (I(N) - I(0)) (Euler for an affine map)."""
    s = maker()
    f = synth.random_occupations(s, 21)
    N = _uneven_bath(s, 22)
    lam = np.random.default_rng(23).normal(size=s.n_states)
    gN = oracle.collision_vjp_nph(s, f, N, lam)
    V = np.random.default_rng(24).normal(size=N.shape)
    h = 0.3
    fd = lam @ (oracle.collision(s, f, N + h * V) - oracle.collision(s, f, N - h * V)) / (2 * h)
    assert fd == pytest.approx(float((gN * V).sum()), rel=1e-11)
    lhs = float((gN * N).sum())
    rhs = float(lam @ (oracle.collision(s, f, N) - oracle.collision(s, f, np.zeros_like(N))))
    assert lhs == pytest.approx(rhs, rel=1e-11)


@pytest.mark.parametrize("maker", [synth.multiband_system, lambda: synth.parabolic_system(4)])
def test_phonon_rate_vjp_finite_differences_and_euler(maker):
    """The phonon-side rate is quadratic in f and affine in N and |g|^2: central
    differences of mu . R are exact up to rounding along any direction; and
    sum_c |g|^2_c dL/d|g|^2_c = mu . R (Euler, R linear in |g|^2)."""
    s = maker()
    f = synth.random_occupations(s, 31)
    N = _uneven_bath(s, 32)
    rng = np.random.default_rng(33)
    mu = rng.normal(size=N.shape)
    gf, gN, gg = oracle.phonon_rate_vjp(s, f, N, mu)
    L = lambda ff, NN, gg2=None: float((mu * oracle.phonon_rate(s, ff, NN, g2=gg2)).sum())
    v = rng.normal(size=s.n_states)
    h = 0.05
    assert (L(f + h * v, N) - L(f - h * v, N)) / (2 * h) == pytest.approx(float(gf @ v), rel=1e-10)
    V = rng.normal(size=N.shape)
    assert (L(f, N + h * V) - L(f, N - h * V)) / (2 * h) == pytest.approx(float((gN * V).sum()), rel=1e-10)
    w = rng.normal(size=s.n_channels) * s.g2
    assert (L(f, N, s.g2 + h * w) - L(f, N, s.g2 - h * w)) / (2 * h) == pytest.approx(float(gg @ w), rel=1e-10)
    assert float(gg @ s.g2) == pytest.approx(L(f, N), rel=1e-11)


def test_coupled_rk4_adjoint_finite_differences():
    """Gradients through two coupled RK4 steps (electrons and phonons) of a
    loss linear in (f_T, N_T), against central differences along random
    directions of f0, of an even direction of N0 and of |g|^2."""
    s = synth.multiband_system()
    f0 = 0.1 + 0.8 * synth.random_occupations(s, 41)
    N0 = s.nph(300.0) * 1.5
    rng = np.random.default_rng(42)
    a = rng.normal(size=s.n_states)
    b = oracle.even_in_q(s, rng.normal(size=N0.shape))
    dt, n = 1.0, 2
    fT, NT, gf, gN, gg = oracle.rk4_coupled_trajectory_grad(s, f0, N0, dt, n, a, b)

    def loss(ff, NN, g2=None):
        for _ in range(n):
            ff, NN = oracle.rk4_coupled_step(s, ff, NN, dt, g2=g2)
        return float(a @ ff + (b * NN).sum())

    assert loss(f0, N0) == pytest.approx(float(a @ fT + (b * NT).sum()), rel=1e-14)
    v = rng.normal(size=s.n_states)
    h = 1e-4
    fd = (loss(f0 + h * v, N0) - loss(f0 - h * v, N0)) / (2 * h)
    assert fd == pytest.approx(float(gf @ v), rel=1e-6)
    V = oracle.even_in_q(s, rng.normal(size=N0.shape))
    fd = (loss(f0, N0 + h * V) - loss(f0, N0 - h * V)) / (2 * h)
    assert fd == pytest.approx(float((gN * V).sum()), rel=1e-6)
    w = rng.normal(size=s.n_channels) * s.g2
    hg = 1e-4     # the difference quotient converges as hg^2 (1e-3 leaves 5e-6)
    fd = (loss(f0, N0, s.g2 + hg * w) - loss(f0, N0, s.g2 - hg * w)) / (2 * hg)
    assert fd == pytest.approx(float(gg @ w), rel=1e-6)


# ---------------------------------------------------------------------------
# Bose statistics: phonon-phonon scattering on the channel list
# ---------------------------------------------------------------------------
def test_bose_two_mode_spontaneous_and_stimulated_decay():
    """Mode 1 sits exactly one third-phonon energy above mode 0.  With one
    quantum in mode 1, mode 0 empty and no third phonons, the golden rule
    gives spontaneous decay 1 -> 0 + phonon at rate C |V|^2 G(0); with m
    quanta already in mode 0 the decay is stimulated by (1 + m) (Bose
    enhancement of the receiving mode), and with N third phonons present the
    emission carries N + 1 while the reverse absorption n_0 N (1 + n_1)
    appears."""
    V2, sig, w = 3e-3, 0.002, 0.02
    s = synth.two_state_system(dE=w, hw=w, g2=V2, sigma=sig, nq=2)
    C = 2 * math.pi / HBAR / 2 * V2 * _G(0.0, sig)
    zero = np.zeros((2, 1))
    I = oracle.collision_bose(s, np.array([0.0, 1.0]), zero)
    assert I[0] == pytest.approx(C, rel=1e-13)
    assert I[1] == pytest.approx(-C, rel=1e-13)
    m = 2.5
    I = oracle.collision_bose(s, np.array([m, 1.0]), zero)
    assert I[1] == pytest.approx(-C * (1 + m), rel=1e-13)
    N = 0.7
    n0, n1 = 0.4, 1.3
    I = oracle.collision_bose(s, np.array([n0, n1]), np.full((2, 1), N))
    expect0 = C * (n1 * (1 + n0) * (N + 1) - n0 * N * (1 + n1))
    assert I[0] == pytest.approx(expect0, rel=1e-12)
    assert I[1] == pytest.approx(-expect0, rel=1e-12)


def test_bose_equilibrium_on_resonant_ladder():
    """Bose-Einstein mode occupations with third phonons at the same
    temperature are a fixed point when every channel is on resonance (the
    counter-process Gaussian underflows): n_p N (1 + n_d) = n_d (1 + n_p)(N + 1)
    for e_d = e_p + w.  Modes hotter than the bath relax (I != 0)."""
    s = synth.ladder_system()
    s.eps = s.eps + 0.01                       # positive mode energies
    nph = s.nph(300.0)
    n_eq = synth.bose_einstein(s.eps, 300.0)
    n_hot = synth.bose_einstein(s.eps, 900.0)
    I_eq = oracle.collision_bose(s, n_eq, nph)
    I_hot = oracle.collision_bose(s, n_hot, nph)
    assert np.abs(I_hot).max() > 0
    assert np.abs(I_eq).max() <= 1e-13 * np.abs(I_hot).max()


def test_bose_conserves_mode_quanta_and_matches_fermi_at_negated_occupations():
    """Every process moves one quantum between the two modes of its channel
    (the third phonon is created or destroyed on its own), so sum_d I_d = 0
    when hw and N are even in q.  Term by term the Bose brackets are minus the
    Fermi brackets of Eq. 2 at f = -n, so collision_bose(n) equals
    -collision(-n), the C oracle written independently."""
    s = synth.ph_ph_system(n=4)
    n = synth.bose_occupations(s, 300.0, seed=8)
    nph = synth.bose_einstein(s.hw, 250.0)
    I = oracle.collision_bose(s, n, nph)
    scale = np.abs(I).max()
    assert scale > 0
    assert abs(I.sum()) <= 1e-13 * scale * math.sqrt(s.n_states)
    assert np.abs(I + oracle.collision(s, -n, nph)).max() <= 1e-13 * scale


def test_bose_vjp_central_differences():
    """collision_bose is quadratic in n and linear in |V|^2 and N, so central
    differences of L = lam . I are exact up to rounding."""
    s = synth.ph_ph_system(n=3)
    rng = np.random.default_rng(12)
    n = synth.bose_occupations(s, 300.0, seed=9)
    nph = synth.bose_einstein(s.hw, 300.0) * (1 + 0.2 * rng.uniform(size=s.hw.shape))
    lam = rng.normal(size=s.n_states)
    gn, gg, gN = oracle.collision_bose_vjp(s, n, nph, lam)
    L = lambda n_, N_, g_: float(lam @ oracle.collision_bose(s, n_, N_, g2=g_))
    for d in rng.choice(s.n_states, 6, replace=False):
        h = 1e-3
        e = np.zeros(s.n_states)
        e[d] = h
        fd = (L(n + e, nph, s.g2) - L(n - e, nph, s.g2)) / (2 * h)
        assert fd == pytest.approx(gn[d], rel=1e-8, abs=1e-10 * np.abs(gn).max())
    for c in rng.choice(s.n_channels, 6, replace=False):
        h = 1e-4 * s.g2[c]
        e = np.zeros(s.n_channels)
        e[c] = h
        fd = (L(n, nph, s.g2 + e) - L(n, nph, s.g2 - e)) / (2 * h)
        assert fd == pytest.approx(gg[c], rel=1e-8, abs=1e-10 * np.abs(gg).max())
    nz = np.argwhere(np.abs(gN) > 1e-6 * np.abs(gN).max())
    for qi, nu in nz[rng.choice(len(nz), 6, replace=False)]:
        h = 1e-3
        e = np.zeros_like(nph)
        e[qi, nu] = h
        fd = (L(n, nph + e, s.g2) - L(n, nph - e, s.g2)) / (2 * h)
        assert fd == pytest.approx(gN[qi, nu], rel=1e-8, abs=1e-10 * np.abs(gN).max())


def test_bose_rk4_trajectory_gradient_finite_differences():
    """The discrete adjoint of RK4 steps of dn/dt = collision_bose(n) against
    central differences of L = g_T . n_T (a polynomial in n0 and |V|^2 of
    degree 2^(4 steps) and 4, so the h^2 truncation is checked to its size)."""
    s = synth.ph_ph_system(n=3)
    rng = np.random.default_rng(14)
    n0 = synth.bose_occupations(s, 300.0, seed=15)
    nph = synth.bose_einstein(s.hw, 300.0)
    gT = rng.normal(size=s.n_states)
    dt, steps = 200.0, 3
    _, gn, gg = oracle.rk4_trajectory_grad(s, n0, nph, dt, steps, gT, statistics="bose")

    def L(n_, g_):
        n = np.array(n_)
        for _ in range(steps):
            n = oracle.rk4_step(s, n, nph, dt, g2=g_, statistics="bose")
        return float(gT @ n)
    for d in rng.choice(s.n_states, 4, replace=False):
        h = 1e-4
        e = np.zeros(s.n_states)
        e[d] = h
        fd = (L(n0 + e, s.g2) - L(n0 - e, s.g2)) / (2 * h)
        assert fd == pytest.approx(gn[d], rel=1e-6, abs=1e-8 * np.abs(gn).max())
    for c in rng.choice(s.n_channels, 4, replace=False):
        h = 1e-3 * s.g2[c]
        e = np.zeros(s.n_channels)
        e[c] = h
        fd = (L(n0, s.g2 + e) - L(n0, s.g2 - e)) / (2 * h)
        assert fd == pytest.approx(gg[c], rel=1e-6, abs=1e-8 * np.abs(gg).max())
