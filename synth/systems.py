"""Seeded synthetic e-ph systems shaped like the paper's workloads.

This module only builds *inputs*: electronic states on a momentum grid
(energies, k indices, velocities), a phonon table (energies per q point and
mode), Bose-Einstein phonon occupations, electron occupations, and the list of
unordered scattering channels (i, j, nu, |g|^2).  It contains none of the
collision-integral arithmetic; both the CPU oracle and the GPU library receive
the arrays it returns.

The paper (Results, "Collision integral, e-ph coupling matrix, and scattering
channels"; Table 1) works with first-principles data we do not have: a few
bands, six phonon modes, 1e4-1e5 window k points and 1e7-1e8 active channels.
The generators below stand in for that data with matched shapes.

Conventions
-----------
* A k point on an (N1, N2, N3) grid has integer coordinates n_a in [0, N_a)
  and linear index (n1*N2 + n2)*N3 + n3.  The same holds for q points on the
  q grid.  Momentum conservation uses commensurate grids: the pair (i, j) is
  allowed when k_j - k_i is a q-grid vector, i.e. divisible by r_a = Nk_a/Nq_a
  in every direction.
* Phonon tables are laid out [Nq][n_modes] (q-major).
* Energies in eV, temperatures in K, velocities in m/s, |g|^2 in eV^2.
* A channel is an unordered state pair (i < j) plus a mode nu; the generator
  emits channels in lexicographic (i, j, nu) order.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os
from typing import Optional

import numpy as np

# CODATA 2018 constants (eV, fs, K, Angstrom).
HBAR_EV_FS = 0.6582119569          # reduced Planck constant, eV*fs
KB_EV_K = 8.617333262e-5           # Boltzmann constant, eV/K
HBAR2_OVER_2ME = 3.80998212        # hbar^2 / (2 m_e), eV*Angstrom^2
LATTICE_A = 5.653                  # Angstrom (GaAs, the paper's first system)

@dataclasses.dataclass
class System:
    """A synthetic e-ph problem.  All arrays are numpy, C-contiguous."""
    name: str
    kgrid: tuple
    qgrid: tuple
    state_k: np.ndarray        # int32 [S], linear k index
    state_band: np.ndarray     # int8  [S]
    eps: np.ndarray            # f64   [S], eV
    n_modes: int
    hw: np.ndarray             # f64   [Nq, n_modes], eV
    ch_i: np.ndarray           # int32 [Nch]
    ch_j: np.ndarray           # int32 [Nch]
    ch_nu: np.ndarray          # int8  [Nch]
    g2: np.ndarray             # f64   [Nch], eV^2
    sigma: float               # Gaussian smearing (standard deviation), eV
    n_q_norm: float            # N_q of the collision integral (full q grid count)
    lattice_a: float = LATTICE_A
    vel: Optional[np.ndarray] = None   # f64 [S, 3], m/s
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_states(self) -> int:
        return int(self.eps.shape[0])

    @property
    def n_channels(self) -> int:
        return int(self.g2.shape[0])

    @property
    def n_q(self) -> int:
        return int(np.prod(self.qgrid))

    def nph(self, T: float) -> np.ndarray:
        """Bose-Einstein phonon occupations [Nq, n_modes] at temperature T."""
        return bose_einstein(self.hw, T)


# --------------------------------------------------------------------------
# counter-based random numbers: splitmix64 (Steele, Lea, Flood, OOPSLA 2014)
# --------------------------------------------------------------------------
def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser applied to the counter x + golden gamma (uint64)."""
    z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _unit_open(u64: np.ndarray) -> np.ndarray:
    """Top 53 bits -> double in (0, 1)."""
    return ((u64 >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def lognormal_g2(key_lo: np.ndarray, key_hi: np.ndarray, nu: np.ndarray, seed: int,
                 median: float = 1e-3, log_sigma: float = 1.0,
                 inv_lo: Optional[np.ndarray] = None,
                 inv_hi: Optional[np.ndarray] = None) -> np.ndarray:
    """|g|^2 = median * exp(log_sigma * Z), Z ~ N(0,1) from Box-Muller on two
    splitmix64 draws keyed by (min id, max id, nu, seed).  Symmetric in the
    pair by construction, so g2(i,j,nu) == g2(j,i,nu).  When the ids of the
    inversion images (k -> -k) are given, the key is the smaller of the pair's
    key and its image's key, so g2 is also inversion symmetric."""
    lo = np.minimum(key_lo, key_hi).astype(np.uint64)
    hi = np.maximum(key_lo, key_hi).astype(np.uint64)
    if inv_lo is not None:
        lo2 = np.minimum(inv_lo, inv_hi).astype(np.uint64)
        hi2 = np.maximum(inv_lo, inv_hi).astype(np.uint64)
        take2 = (lo2 < lo) | ((lo2 == lo) & (hi2 < hi))
        lo = np.where(take2, lo2, lo)
        hi = np.where(take2, hi2, hi)
    key = (lo << np.uint64(26)) ^ hi
    key = (key << np.uint64(3)) ^ np.asarray(nu, dtype=np.uint64)
    salt = (int(seed) * 0x2545F4914F6CDD1D) & 0xFFFFFFFFFFFFFFFF
    key ^= splitmix64(np.array([salt], dtype=np.uint64))[0]
    key <<= np.uint64(1)
    u1 = _unit_open(splitmix64(key))
    u2 = _unit_open(splitmix64(key | np.uint64(1)))
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    return median * np.exp(log_sigma * z)


# --------------------------------------------------------------------------
# occupations
# --------------------------------------------------------------------------
def fermi_dirac(eps: np.ndarray, mu: float, T: float) -> np.ndarray:
    x = (np.asarray(eps, dtype=np.float64) - mu) / (KB_EV_K * T)
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def bose_einstein(hw: np.ndarray, T: float) -> np.ndarray:
    hw = np.asarray(hw, dtype=np.float64)
    out = np.zeros_like(hw)
    ok = hw > 0
    out[ok] = 1.0 / np.expm1(hw[ok] / (KB_EV_K * T))
    return out


# --------------------------------------------------------------------------
# grids and phonons
# --------------------------------------------------------------------------
def grid_coords(grid) -> np.ndarray:
    """Integer coordinates [N, 3] of every point of a grid, in linear order."""
    g = [np.arange(n) for n in grid]
    c = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    return c.astype(np.int64)


def linear_index(coords: np.ndarray, grid) -> np.ndarray:
    c = np.asarray(coords, dtype=np.int64)
    return (c[..., 0] * grid[1] + c[..., 1]) * grid[2] + c[..., 2]


def minimal_image_frac(coords: np.ndarray, grid) -> np.ndarray:
    """Fractional coordinates folded into [-1/2, 1/2), via the integer minimal
    image so that c and N - c give values of exactly opposite sign."""
    c = np.asarray(coords, dtype=np.int64)
    n = np.asarray(grid, dtype=np.int64)
    m = (c + n // 2) % n - n // 2
    return m.astype(np.float64) / n.astype(np.float64)


def phonon_table(qgrid, a: float, debye_speeds_kms=(), einstein_eV=()) -> np.ndarray:
    """hw [Nq, n_modes]: Debye modes hbar*c*|q| with |q| the minimal-image
    Cartesian length on a simple-cubic reciprocal lattice, then Einstein modes."""
    qc = grid_coords(qgrid)
    qcart = minimal_image_frac(qc, qgrid) * (2.0 * math.pi / a)    # 1/Angstrom
    qlen = np.sqrt((qcart ** 2).sum(axis=1))
    cols = []
    for c in debye_speeds_kms:
        c_ang_fs = c * 1e3 * 1e10 / 1e15                            # Angstrom/fs
        cols.append(HBAR_EV_FS * c_ang_fs * qlen)
    for w in einstein_eV:
        cols.append(np.full(qlen.shape, float(w)))
    return np.ascontiguousarray(np.stack(cols, axis=1))


def inverse_k(state_k: np.ndarray, kgrid) -> np.ndarray:
    """Linear index of -k for every k."""
    kc = grid_coords(kgrid)[np.asarray(state_k, dtype=np.int64)]
    return linear_index((-kc) % np.asarray(kgrid), kgrid)


def q_of_pair(kc_i: np.ndarray, kc_j: np.ndarray, kgrid, qgrid) -> np.ndarray:
    """Linear q index of k_j - k_i (commensurate pairs only)."""
    kg = np.asarray(kgrid, dtype=np.int64)
    r = kg // np.asarray(qgrid, dtype=np.int64)
    d = (np.asarray(kc_j, dtype=np.int64) - np.asarray(kc_i, dtype=np.int64)) % kg
    assert np.all(d % r == 0), "pair is not commensurate with the q grid"
    return linear_index(d // r, qgrid)


# --------------------------------------------------------------------------
# channel enumeration
# --------------------------------------------------------------------------
def enumerate_channels(state_k, kgrid, qgrid, hw, key_ids, seed,
                       pair_filter=None, hw_min=1e-6, inv_key_ids=None):
    """All unordered commensurate pairs (i < j) times all modes whose phonon
    energy is at least hw_min, in lexicographic (i, j, nu) order.

    States must be ordered so that each commensurability class (coset of the
    q grid inside the k grid) is contiguous; the caller's state order is kept.
    pair_filter(i, j) -> bool mask may drop pairs (energy cutoffs)."""
    kgrid = tuple(int(x) for x in kgrid)
    qgrid = tuple(int(x) for x in qgrid)
    kc = grid_coords(kgrid)[np.asarray(state_k, dtype=np.int64)]
    r = np.asarray(kgrid) // np.asarray(qgrid)
    coset = linear_index(kc % r, tuple(int(x) for x in r))
    assert _contiguous_classes(coset), "states of one coset must be contiguous"
    n_modes = hw.shape[1]
    tasks = []
    for c in _class_order(coset):
        idx = np.nonzero(coset == c)[0]
        n = idx.size
        # rows of the upper triangle, chunked so temporaries stay small
        row_chunk = max(1, int(4_000_000 // max(n, 1)))
        for r0 in range(0, n - 1, row_chunk):
            tasks.append((idx, r0, min(n - 1, r0 + row_chunk)))

    def work(task):
        idx, r0, r1 = task
        ii, jj = _triu_rows(r0, r1, idx.size)
        si, sj = idx[ii], idx[jj]
        if pair_filter is not None:
            keep = pair_filter(si, sj)
            si, sj = si[keep], sj[keep]
        q = q_of_pair(kc[si], kc[sj], kgrid, qgrid)
        ok = hw[q] >= hw_min                            # [npairs, n_modes]
        pi = np.broadcast_to(si[:, None], ok.shape)[ok]
        pj = np.broadcast_to(sj[:, None], ok.shape)[ok]
        pn = np.broadcast_to(np.arange(n_modes)[None, :], ok.shape)[ok]
        inv = (None, None) if inv_key_ids is None else (inv_key_ids[pi], inv_key_ids[pj])
        return (pi.astype(np.int32), pj.astype(np.int32), pn.astype(np.int8),
                lognormal_g2(key_ids[pi], key_ids[pj], pn, seed, inv_lo=inv[0], inv_hi=inv[1]))

    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(work, tasks))
    cat = (lambda k, dt: np.concatenate([p[k] for p in parts]).astype(dt, copy=False)
           if parts else np.zeros(0, dtype=dt))
    ch_i, ch_j = cat(0, np.int32), cat(1, np.int32)
    ch_nu, g2 = cat(2, np.int8), cat(3, np.float64)
    # rows ascend inside a class and classes follow state order, so the list
    # is lexicographic by construction; spot-check it on small problems
    if ch_i.size < 5_000_000:
        assert _is_lex_sorted(ch_i, ch_j, ch_nu)
    return ch_i, ch_j, ch_nu, g2


def _triu_rows(r0, r1, n):
    rows = np.arange(r0, r1)
    counts = n - 1 - rows
    ii = np.repeat(rows, counts)
    start = np.repeat(np.cumsum(counts) - counts, counts)
    jj = np.arange(ii.size) - start + np.repeat(rows + 1, counts)
    return ii, jj


def _contiguous_classes(c):
    change = np.nonzero(np.diff(c) != 0)[0]
    seen = c[np.concatenate([[0], change + 1])]
    return len(seen) == len(np.unique(seen))


def _class_order(c):
    change = np.nonzero(np.diff(c) != 0)[0]
    return list(c[np.concatenate([[0], change + 1])]) if c.size else []


def _is_lex_sorted(i, j, nu):
    key = (i.astype(np.int64) << 33) | (j.astype(np.int64) << 3) | nu.astype(np.int64)
    return bool(np.all(np.diff(key) > 0))


# --------------------------------------------------------------------------
# systems
# --------------------------------------------------------------------------
def parabolic_system(n=8, m_eff=0.3, a=LATTICE_A, debye_kms=(5.0,), einstein_eV=(0.030, 0.050),
                     sigma=0.008, seed=2511, name=None) -> System:
    """One parabolic band eps = hbar^2 |k|^2 / (2 m* m_e) on an n^3 grid with
    the q grid equal to the k grid; every state is kept and every pair is a
    channel (no energy or |g| cutoff).  n=8 is the 512-k test case."""
    kgrid = (n, n, n)
    kc = grid_coords(kgrid)
    kcart = minimal_image_frac(kc, kgrid) * (2.0 * math.pi / a)
    eps = (HBAR2_OVER_2ME / m_eff) * (kcart ** 2).sum(axis=1)
    hw = phonon_table(kgrid, a, debye_kms, einstein_eV)
    state_k = np.arange(kc.shape[0], dtype=np.int32)
    ch = enumerate_channels(state_k, kgrid, kgrid, hw, state_k.astype(np.int64), seed,
                            inv_key_ids=inverse_k(state_k, kgrid))
    vel = (kcart * (2.0 * HBAR2_OVER_2ME / m_eff) / HBAR_EV_FS) * 1e5   # Angstrom/fs -> m/s
    return System(name=name or f"parabolic{n}", kgrid=kgrid, qgrid=kgrid, state_k=state_k,
                  state_band=np.zeros(state_k.size, np.int8), eps=eps, n_modes=hw.shape[1],
                  hw=hw, ch_i=ch[0], ch_j=ch[1], ch_nu=ch[2], g2=ch[3], sigma=sigma,
                  n_q_norm=float(np.prod(kgrid)), lattice_a=a, vel=vel,
                  meta=dict(m_eff=m_eff, seed=seed))


def c1_occupations(system: System, mu=0.25, T=300.0, pert_seed=3683, amp=0.1) -> np.ndarray:
    """Fermi-Dirac occupations times (1 + amp*u), u ~ U[-1, 1], clipped to [0, 1]."""
    rng = np.random.Generator(np.random.Philox(pert_seed))
    u = rng.uniform(-1.0, 1.0, size=system.n_states)
    return np.clip(fermi_dirac(system.eps, mu, T) * (1.0 + amp * u), 0.0, 1.0)


def random_occupations(system: System, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.Philox(seed))
    return rng.uniform(0.0, 1.0, size=system.n_states)


def two_state_system(dE=0.05, hw=0.05, g2=2e-3, sigma=0.004, nq=2) -> System:
    """Two states on a 2x1x1 grid joined by one channel with one dispersionless mode."""
    kgrid = (nq, 1, 1)
    hwt = np.full((nq, 1), float(hw))
    return System(name="two_state", kgrid=kgrid, qgrid=kgrid,
                  state_k=np.array([0, 1], np.int32), state_band=np.zeros(2, np.int8),
                  eps=np.array([0.0, dE]), n_modes=1, hw=hwt,
                  ch_i=np.array([0], np.int32), ch_j=np.array([1], np.int32),
                  ch_nu=np.array([0], np.int8), g2=np.array([float(g2)]),
                  sigma=sigma, n_q_norm=float(nq))


def field_drift_rates(E_V_per_m, kgrid, a=LATTICE_A, charge=-1.0) -> np.ndarray:
    """Per-axis drift rates r_a = F_a / (hbar dk_a) in 1/fs for an electric field
    E (V/m) on a simple-cubic k grid of lattice constant a (Angstrom):
    F = charge * e * E in eV/Angstrom, dk_a = 2 pi / (a N_a) in 1/Angstrom."""
    E = np.asarray(E_V_per_m, np.float64)
    F = charge * E * 1e-10
    dk = 2.0 * math.pi / (a * np.asarray(kgrid, np.float64))
    return F / (HBAR_EV_FS * dk)


def defect_system(n=6, with_phonons=True, defect_median=2e-3, seed=2511) -> System:
    """Parabolic band on an n^3 grid with one elastic (e-defect) mechanism as
    an extra mode of zero energy: every pair of states is coupled through it,
    |g|^2 lognormal with median defect_median.  With with_phonons the phonon
    channels of parabolic_system(n) are kept beside it.  The elastic mode is
    the last one (bit n_modes - 1 of the elastic mask); nph(T) gives it N = 0."""
    base = parabolic_system(n, seed=seed)
    S = base.n_states
    hw = np.concatenate([base.hw, np.zeros((base.hw.shape[0], 1))], axis=1)
    nu_e = hw.shape[1] - 1
    ii, jj = np.triu_indices(S, 1)
    ii, jj = ii.astype(np.int32), jj.astype(np.int32)
    nu = np.full(ii.size, nu_e, np.int8)
    g2 = lognormal_g2(ii, jj, nu, seed + 17, median=defect_median)
    if with_phonons:
        ci = np.concatenate([base.ch_i, ii])
        cj = np.concatenate([base.ch_j, jj])
        cn = np.concatenate([base.ch_nu, nu])
        cg = np.concatenate([base.g2, g2])
        order = np.lexsort((cn, cj, ci))
        ci, cj, cn, cg = ci[order], cj[order], cn[order], cg[order]
    else:
        ci, cj, cn, cg = ii, jj, nu, g2
    return System(name=f"defect{n}", kgrid=base.kgrid, qgrid=base.qgrid, state_k=base.state_k,
                  state_band=base.state_band, eps=base.eps, n_modes=hw.shape[1], hw=hw,
                  ch_i=ci.astype(np.int32), ch_j=cj.astype(np.int32), ch_nu=cn.astype(np.int8),
                  g2=cg, sigma=base.sigma, n_q_norm=base.n_q_norm, lattice_a=base.lattice_a,
                  vel=base.vel, meta=dict(base.meta, elastic_mode=nu_e))


def ladder_system(n_rungs=6, per_rung=8, hw_e=0.050, sigma=0.002, seed=7) -> System:
    """Resonant ladder: state energies sit exactly on rungs n*hw_e, one
    dispersionless mode of energy hw_e, and channels only between adjacent rungs.
    The counter-process Gaussian is then exp(-(2 hw_e)^2 / (2 sigma^2)), which
    underflows to zero, so detailed balance holds channel by channel."""
    S = n_rungs * per_rung
    n = 1
    while n ** 3 < S:
        n += 1
    kgrid = (n, n, n)
    rng = np.random.Generator(np.random.Philox(seed))
    state_k = np.sort(rng.choice(n ** 3, size=S, replace=False)).astype(np.int32)
    rung = np.repeat(np.arange(n_rungs), per_rung)
    rng.shuffle(rung)
    eps = rung * hw_e
    hw = np.full((n ** 3, 1), hw_e)
    ii, jj = np.triu_indices(S, 1)
    keep = np.abs(rung[ii] - rung[jj]) == 1
    ii, jj = ii[keep].astype(np.int32), jj[keep].astype(np.int32)
    nu = np.zeros(ii.size, np.int8)
    g2 = lognormal_g2(ii, jj, nu, seed)
    return System(name="ladder", kgrid=kgrid, qgrid=kgrid, state_k=state_k,
                  state_band=np.zeros(S, np.int8), eps=eps.astype(np.float64), n_modes=1,
                  hw=hw, ch_i=ii, ch_j=jj, ch_nu=nu, g2=g2, sigma=sigma,
                  n_q_norm=float(n ** 3), meta=dict(rung=rung))


def random_channel_system(n_states=40, n_channels=300, kn=4, n_modes=3, sigma=0.02,
                          seed=11, e_max=0.3) -> System:
    """Small unstructured problem: random states on a kn^3 grid (q grid = k
    grid, one state per k point), random unordered pairs, arbitrary channel
    order, i and j given in either orientation.  Used for layout edge cases."""
    rng = np.random.Generator(np.random.Philox(seed))
    kgrid = (kn, kn, kn)
    S = min(n_states, kn ** 3)
    state_k = rng.choice(kn ** 3, size=S, replace=False).astype(np.int32)
    eps = rng.uniform(0.0, e_max, size=S)
    h = rng.uniform(0.005, 0.06, size=(kn ** 3, n_modes))
    minus_q = inverse_k(np.arange(kn ** 3), kgrid)
    hw = 0.5 * (h + h[minus_q])                      # even in q, as time reversal requires
    ci = rng.integers(0, S, size=n_channels)
    cj = rng.integers(0, S - 1, size=n_channels)
    cj = np.where(cj >= ci, cj + 1, cj)
    nu = rng.integers(0, n_modes, size=n_channels).astype(np.int8)
    # drop repeated (unordered pair, mode) draws, keeping the first occurrence
    key = (np.minimum(ci, cj) * S + np.maximum(ci, cj)) * 8 + nu
    _, first = np.unique(key, return_index=True)
    keep = np.sort(first)
    ci, cj, nu = ci[keep], cj[keep], nu[keep]
    g2 = lognormal_g2(ci, cj, nu, seed)
    return System(name="random", kgrid=kgrid, qgrid=kgrid, state_k=state_k,
                  state_band=np.zeros(S, np.int8), eps=eps, n_modes=n_modes, hw=hw,
                  ch_i=ci.astype(np.int32), ch_j=cj.astype(np.int32), ch_nu=nu, g2=g2,
                  sigma=sigma, n_q_norm=float(kn ** 3))


# --------------------------------------------------------------------------
# tight-binding cubic model (the 100^3 / 50^3, six-mode transport workload)
# --------------------------------------------------------------------------
def _tb_matrices(seed, nb):
    rng = np.random.Generator(np.random.Philox(seed))
    def sym(scale):
        m = rng.normal(0.0, scale, size=(nb, nb))
        return 0.5 * (m + m.T)
    H0 = sym(1.0) + np.diag(np.linspace(0.0, 3.0, nb))
    T = sym(0.5)
    U = sym(0.2)
    return H0, T, U


def _tb_hamiltonian(cos3, H0, T, U):
    c = cos3
    s1 = c.sum(axis=1)
    s2 = c[:, 0] * c[:, 1] + c[:, 0] * c[:, 2] + c[:, 1] * c[:, 2]
    return H0[None] + 2.0 * s1[:, None, None] * T[None] + 2.0 * s2[:, None, None] * U[None]


def tb_system(kn=100, qn=50, nb=4, target_states=23000, window=0.3, a=LATTICE_A,
              debye_kms=(5.0, 3.0, 3.0), einstein_eV=(0.020, 0.040, 0.060), sigma=0.008,
              seed=2511, energy_cutoff=None, name=None, with_channels=True) -> System:
    """Random real-symmetric nb-band tight-binding model with cubic symmetry,
    H(k) = H0 + 2T sum_a cos(k_a a) + 2U sum_{a<b} cos(k_a a) cos(k_b a), scaled so
    that about target_states states lie within `window` eV of the global
    minimum.  States are ordered by (q-grid coset, k, band).  Channels: every
    commensurate pair of window states, all band pairs and modes; an optional
    energy_cutoff = (n_sigma,) keeps a pair only if min_nu |de -/+ hw| < n_sigma*sigma."""
    kgrid = (kn, kn, kn)
    qgrid = (qn, qn, qn)
    H0, T, U = _tb_matrices(seed, nb)
    # eigenvalues on the full grid, in slabs to bound memory
    # minimal-image angles, so that H(k) and H(-k) are bitwise equal and the
    # window keeps whole inversion pairs
    ang = 2.0 * math.pi * minimal_image_frac(np.arange(kn), kn)
    cs = np.cos(ang)
    evals = np.empty((kn ** 3, nb))
    slab = kn * kn
    c_yz = np.stack(np.meshgrid(cs, cs, indexing="ij"), -1).reshape(-1, 2)
    for x in range(kn):
        cos3 = np.column_stack([np.full(slab, cs[x]), c_yz])
        evals[x * slab:(x + 1) * slab] = np.linalg.eigvalsh(_tb_hamiltonian(cos3, H0, T, U))
    emin = evals.min()
    flat = np.sort((evals - emin).ravel())
    t = flat[min(target_states, flat.size) - 1]
    scale = window / t
    e_all = (evals - emin) * scale
    sel_k, sel_b = np.nonzero(e_all <= window)
    kc = grid_coords(kgrid)[sel_k]
    r = kn // qn
    coset = linear_index(kc % r, (r, r, r))
    order = np.lexsort((sel_b, sel_k, coset))
    sel_k, sel_b = sel_k[order], sel_b[order]
    kc = kc[order]
    eps = e_all[sel_k, sel_b]
    # velocities by Hellmann-Feynman on the selected states
    ka = minimal_image_frac(kc, kgrid) * (2.0 * math.pi)
    cos3, sin3 = np.cos(ka), np.sin(ka)
    Hs = _tb_hamiltonian(cos3, H0, T, U)
    w_, vecs = np.linalg.eigh(Hs)
    u = vecs[np.arange(sel_b.size), :, sel_b]                   # [S, nb]
    vel = np.empty((sel_b.size, 3))
    for al in range(3):
        others = [b for b in range(3) if b != al]
        dcos = -a * sin3[:, al]                                # d cos(k_a a) / dk_a
        dH = 2.0 * dcos[:, None, None] * (T[None] + U[None] * (cos3[:, others[0]] + cos3[:, others[1]])[:, None, None])
        vel[:, al] = np.einsum("si,sij,sj->s", u, dH, u) * scale / HBAR_EV_FS * 1e5
    hw = phonon_table(qgrid, a, debye_kms, einstein_eV)
    state_k = linear_index(kc, kgrid).astype(np.int32)
    key_ids = state_k.astype(np.int64) * nb + sel_b
    inv_ids = inverse_k(state_k, kgrid) * nb + sel_b
    if not with_channels:
        z = np.zeros(0, np.int32)
        return System(name=name or f"tb{kn}-states", kgrid=kgrid, qgrid=qgrid, state_k=state_k,
                      state_band=sel_b.astype(np.int8), eps=eps, n_modes=hw.shape[1], hw=hw,
                      ch_i=z, ch_j=z.copy(), ch_nu=np.zeros(0, np.int8), g2=np.zeros(0),
                      sigma=sigma, n_q_norm=float(qn ** 3), lattice_a=a, vel=vel,
                      meta=dict(seed=seed, scale_eV=scale, window=window, nb=nb,
                                key_ids=key_ids, inv_ids=inv_ids))
    pair_filter = None
    if energy_cutoff is not None:
        n_sig = float(energy_cutoff)
        w_max = float(hw.max())
        def pair_filter(si, sj):
            de = np.abs(eps[si] - eps[sj])
            return (de < w_max + n_sig * sigma)
    ch = enumerate_channels(state_k, kgrid, qgrid, hw, key_ids, seed, pair_filter=pair_filter,
                            inv_key_ids=inv_ids)
    if energy_cutoff is not None and ch[0].size:
        q = q_of_pair(kc[ch[0]], kc[ch[1]], kgrid, qgrid)
        w = hw[q, ch[2].astype(np.int64)]
        de = eps[ch[0]] - eps[ch[1]]
        keep = np.minimum(np.abs(de + w), np.abs(de - w)) < float(energy_cutoff) * sigma
        ch = tuple(x[keep] for x in ch)
    return System(name=name or f"tb{kn}", kgrid=kgrid, qgrid=qgrid, state_k=state_k,
                  state_band=sel_b.astype(np.int8), eps=eps, n_modes=hw.shape[1], hw=hw,
                  ch_i=ch[0], ch_j=ch[1], ch_nu=ch[2], g2=ch[3], sigma=sigma,
                  n_q_norm=float(qn ** 3), lattice_a=a, vel=vel,
                  meta=dict(seed=seed, scale_eV=scale, window=window, nb=nb,
                            energy_cutoff=energy_cutoff))


def tb_two_band_system(**kw) -> System:
    """The tight-binding transport workload's model with a seed (124) whose
    0.3 eV window holds two bands: 15,544 states of the lowest band and 7,465
    of the next, 23,009 in all, 1.98e8 channels (intra- and inter-band pairs;
    pairs at the same k have no acoustic channel, q = 0)."""
    kw.setdefault("seed", 124)
    kw.setdefault("name", "tb100_2band")
    return tb_system(**kw)


def ph_ph_system(n=6, a=LATTICE_A, debye_kms=(4.0, 7.0), einstein_eV=(0.030,), sigma=0.002,
                 hw_min=1e-3, v2_scale=1e-4, seed=31, name=None) -> System:
    """Phonon-phonon (three-phonon) scattering on the channel-list layout
    (Bose plans): the states are the phonon modes (q, branch) of an n^3 grid
    with hbar omega >= hw_min (the acoustic modes at q = 0 are left out), with
    energies from the same Debye/Einstein model as the e-ph systems; a
    channel (i, j, nu) couples modes i and j through the third phonon of
    branch nu at q = q_j - q_i, whose energy is the table hw of the same
    model.  Every pair and third branch with hbar omega >= hw_min is a
    channel; |V3|^2 is the seeded lognormal of the e-ph systems times
    v2_scale (a stand-in, not anharmonic data, scaled so that the modes relax
    over picoseconds, as phonons do, rather than over the femtoseconds of
    electrons)."""
    qgrid = (n, n, n)
    hw = phonon_table(qgrid, a, debye_kms, einstein_eV)
    nq, nb = hw.shape
    qi, bi = np.meshgrid(np.arange(nq), np.arange(nb), indexing="ij")
    keep = hw[qi, bi] >= hw_min
    state_k = qi[keep].astype(np.int32)
    band = bi[keep].astype(np.int8)
    eps = hw[qi, bi][keep].astype(np.float64)
    key = (state_k.astype(np.int64) * nb + band).astype(np.int64)
    ch = enumerate_channels(state_k, qgrid, qgrid, hw, key, seed, hw_min=hw_min)
    return System(name=name or f"phph{n}", kgrid=qgrid, qgrid=qgrid, state_k=state_k, state_band=band,
                  eps=eps, n_modes=nb, hw=hw, ch_i=ch[0], ch_j=ch[1], ch_nu=ch[2], g2=ch[3] * v2_scale,
                  sigma=sigma,
                  n_q_norm=float(nq), lattice_a=a, meta=dict(seed=seed, statistics="bose"))


def bose_occupations(system: System, T: float = 300.0, seed: int = 5, amp: float = 0.3) -> np.ndarray:
    """Bose-Einstein occupations of the modes at T, each scaled by a seeded
    factor in [1 - amp, 1 + amp] (out of equilibrium)."""
    rng = np.random.default_rng(seed)
    return bose_einstein(np.asarray(system.eps, np.float64), T) * (1.0 + amp * (2.0 * rng.uniform(size=system.n_states) - 1.0))


def multiband_system(kn=6, qn=3, nb=2, n_k=24, e_max=0.25, a=LATTICE_A,
                     debye_kms=(4.0,), einstein_eV=(0.02, 0.045), sigma=0.015,
                     seed=19) -> System:
    """Tiny multi-band problem on commensurate grids with the q grid coarser
    than the k grid (r = kn/qn): n_k random k points, nb bands each with random
    energies, states ordered by (coset, k, band); every commensurate pair and
    mode is a channel except acoustic modes at q = 0 (hw = 0)."""
    rng = np.random.Generator(np.random.Philox(seed))
    kgrid, qgrid = (kn,) * 3, (qn,) * 3
    ks = np.sort(rng.choice(kn ** 3, size=n_k, replace=False))
    kc = grid_coords(kgrid)[ks]
    r = kn // qn
    coset = linear_index(kc % r, (r, r, r))
    order = np.lexsort((ks, coset))
    ks = ks[order]
    state_k = np.repeat(ks, nb).astype(np.int32)
    band = np.tile(np.arange(nb), ks.size).astype(np.int8)
    eps = rng.uniform(0.0, e_max, size=state_k.size)
    hw = phonon_table(qgrid, a, debye_kms, einstein_eV)
    key_ids = state_k.astype(np.int64) * nb + band
    ch = enumerate_channels(state_k, kgrid, qgrid, hw, key_ids, seed)
    return System(name="multiband", kgrid=kgrid, qgrid=qgrid, state_k=state_k,
                  state_band=band, eps=eps, n_modes=hw.shape[1], hw=hw,
                  ch_i=ch[0], ch_j=ch[1], ch_nu=ch[2], g2=ch[3], sigma=sigma,
                  n_q_norm=float(qn ** 3), lattice_a=a)


def parabolic_states(n=60, a=20.0, m_eff=0.3) -> tuple:
    """States only (no channels) of one parabolic band on an n^3 grid:
    returns (eps [S] eV, vel [S,3] m/s)."""
    kc = grid_coords((n, n, n))
    kcart = minimal_image_frac(kc, (n, n, n)) * (2.0 * math.pi / a)
    eps = (HBAR2_OVER_2ME / m_eff) * (kcart ** 2).sum(axis=1)
    vel = (kcart * (2.0 * HBAR2_OVER_2ME / m_eff) / HBAR_EV_FS) * 1e5
    return eps, vel


def pulse_occupations(system: System, mu=-0.1, T=300.0, amplitude=0.1, center=0.2,
                      width=0.05) -> np.ndarray:
    """Fermi-Dirac background plus a Gaussian electron pulse:
    f = FD(eps; mu, T) + amplitude * exp(-(eps - center)^2 / (2 width^2)), clipped to [0, 1]."""
    e = np.asarray(system.eps, dtype=np.float64)
    f = fermi_dirac(e, mu, T) + amplitude * np.exp(-0.5 * ((e - center) / width) ** 2)
    return np.clip(f, 0.0, 1.0)


def batch_occupations(system: System, mu=0.05, temps=None, fields=None, tau0_fs=10.0) -> np.ndarray:
    """A family of electron occupation vectors, one per (temperature, field):
    Fermi-Dirac at T_b displaced by a field E_b along x,
    f_b(s) = FD(eps_s + tau0 e E_b v_x(s); mu, T_b), with tau0 e E_b v_x in eV
    for E in V/m, tau0 in fs and v in m/s.  Default: 16 temperatures from
    100 to 400 K times 4 fields from 0 to 1e5 V/m (64 rows, temperature-major)."""
    temps = np.linspace(100.0, 400.0, 16) if temps is None else np.asarray(temps, dtype=np.float64)
    fields = np.linspace(0.0, 1e5, 4) if fields is None else np.asarray(fields, dtype=np.float64)
    vx = np.asarray(system.vel, dtype=np.float64)[:, 0]
    rows = []
    for T in temps:
        for Ef in fields:
            shift = tau0_fs * 1e-15 * Ef * vx
            rows.append(fermi_dirac(np.asarray(system.eps) + shift, mu, T))
    return np.stack(rows)


def grouped_system(n_systems=16, ch_min=1e5, ch_max=1e7, seed=2511, base=None) -> System:
    """Uneven batch of small systems in one problem: n_systems subsets of the
    tight-binding window states (each inside one coset of the q grid, so every
    pair is commensurate), with channel counts log-spaced from ch_min to
    ch_max.  Each subset keeps all its pairs and modes; subsets share no
    states and no channels (a block-diagonal channel list), and share the
    phonon table.  meta['offsets'] holds each subsystem's state range and
    meta['ch_offsets'] its channel range."""
    base = base or tb_system(seed=seed, with_channels=False)
    kc = grid_coords(base.kgrid)[base.state_k]
    r = np.asarray(base.kgrid) // np.asarray(base.qgrid)
    coset = linear_index(kc % r, tuple(int(x) for x in r))
    rng = np.random.Generator(np.random.Philox(seed + 7))
    targets = np.geomspace(ch_min, ch_max, n_systems)
    nm = base.n_modes
    parts, offs, choffs = [], [0], [0]
    ci_l, cj_l, cn_l, g_l = [], [], [], []
    for m, tgt in enumerate(targets):
        n = int(round((1 + np.sqrt(1 + 8 * tgt / nm)) / 2))
        c = m % int(coset.max() + 1)
        pool = np.nonzero(coset == c)[0]
        n = min(n, pool.size)
        idx = np.sort(rng.choice(pool, size=n, replace=False))
        sk = base.state_k[idx]
        ids = np.asarray(base.meta["key_ids"])[idx] * 64 + m
        inv = np.asarray(base.meta["inv_ids"])[idx] * 64 + m
        ch = enumerate_channels(sk, base.kgrid, base.qgrid, base.hw, ids, seed + m,
                                inv_key_ids=inv)
        ci_l.append(ch[0] + offs[-1])
        cj_l.append(ch[1] + offs[-1])
        cn_l.append(ch[2])
        g_l.append(ch[3])
        parts.append(idx)
        offs.append(offs[-1] + n)
        choffs.append(choffs[-1] + ch[0].size)
    idx = np.concatenate(parts)
    return System(name=f"grouped{n_systems}", kgrid=base.kgrid, qgrid=base.qgrid,
                  state_k=base.state_k[idx].astype(np.int32), state_band=base.state_band[idx],
                  eps=base.eps[idx], n_modes=nm, hw=base.hw,
                  ch_i=np.concatenate(ci_l).astype(np.int32), ch_j=np.concatenate(cj_l).astype(np.int32),
                  ch_nu=np.concatenate(cn_l).astype(np.int8), g2=np.concatenate(g_l),
                  sigma=base.sigma, n_q_norm=base.n_q_norm, lattice_a=base.lattice_a,
                  vel=base.vel[idx], meta=dict(offsets=offs, ch_offsets=choffs,
                                                targets=targets.tolist()))
