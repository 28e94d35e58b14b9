"""FP64 CPU oracle for the e-ph collision integral and its consumers.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
cpu_baseline leg may import this package.  It shares no code with the GPU
library (paper_2511_03683_amd): it has its own C file (eph_oracle.c), its own
constants and its own q-index, Gaussian and occupation-factor arithmetic.

Contents, each following the paper (arXiv 2511.03683):

* select_channels(sys, ...)     -- the channel selection that precedes the
  list (scattering-channel paragraph after Eq. 2: approximate energy
  conservation with the Gaussian delta, a cutoff on |g|), as a keep mask.
* collision_elastic(sys, f)     -- the elastic (e-defect) golden rule over
  the channels of given mechanisms (Discussion: other scattering mechanisms
  on the same data structure), written out in numpy.
* collision(sys, f, nph)        -- Eq. 2 over a channel list (Results,
  "Collision integral ..."; the channel-list loop is the Baseline-CPU loop
  shape of "Reference CPU algorithm", run sequentially).
* collision_threads(sys, f, nph) -- the same C loop over disjoint slices of
  the list on several host threads, partial vectors added in slice order
  (the multi-core Baseline-CPU shape without atomics).
* collision_brute(sys, f, nph)  -- Eq. 2 written out over the full q grid,
  all bands and modes, for tiny grids (numpy; independent of the C code).
* collision_vjp(...)            -- hand-derived reverse mode of Eq. 2.
* collision_bose(sys, n, nph), collision_bose_vjp(...) -- the same golden
  rule with Bose factors (1 + n) for phonon modes as the states: three-phonon
  scattering on the channel list (Discussion: other mechanisms on the same
  data structure), written out in numpy, and its hand-derived reverse mode.
* phonon_rate(sys, f, nph)      -- dN/dt of every phonon (q, mode) from the
  same channel list: the phonon side of the four golden-rule processes
  behind Eq. 2 (coupled electron-phonon dynamics; the paper cites it, the
  formula is the reading documented with the function).
* drift(sys, f, rates)          -- the field term of Eq. 1, -(1/hbar) F . grad_k f,
  by central differences on the k grid (the discretisation is a reading:
  the paper defers it to its Methods), and its transpose.
* rk4_step / rk4_adjoint_step   -- classical RK4 for df/dt = I[f] (the
  paper's real-time BTE; the integrator is not named in the text, RK4 is the
  reading adopted here) and its exact discrete adjoint, with the drift term
  when rates are given.
* rk4_coupled_step, even_in_q   -- electrons and phonons stepped together,
  the phonons of q and -q as a pair (even part of the rate).
* collision_vjp_nph, phonon_rate_vjp, rk4_coupled_adjoint_step,
  rk4_coupled_trajectory_grad   -- reverse mode with respect to the phonon
  occupations, of the phonon-side rate, and of the coupled RK4 step (the
  exact discrete adjoint of the computed steps), derived by hand.
* transport_*                   -- linearised steady-state BTE (Eq. 1 with the
  collision integral linearised at f0), iterated to self-consistency.

Parity status: every function here is pinned by tests/test_oracle.py
(closed forms, invariants, brute force, finite differences); the absolute
physics of the paper's materials is "parity unpinned" (no data).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

HBAR_EV_FS = 0.6582119569
KB_EV_K = 8.617333262e-5


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        common = [ctypes.c_int, P, P, P, P, ctypes.c_int, P, P, ctypes.c_double,
                  ctypes.c_double, ctypes.c_int64, P, P, P, P]
        lib.orc_collision.argtypes = common + [P, P, P]
        lib.orc_collision.restype = None
        lib.orc_collision_vjp.argtypes = common + [P, P, P, P]
        lib.orc_collision_vjp.restype = None
        lib.orc_transport_coeffs.argtypes = common + [P, P, P, P]
        lib.orc_transport_coeffs.restype = None
        lib.orc_collision_inout.argtypes = common + [P, P, P]
        lib.orc_collision_inout.restype = None
        _LIB = lib
    return _LIB


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Args:
    """Holds contiguous copies of a system's arrays for the C calls."""

    def __init__(self, sys, nph, g2=None):
        self.S = sys.n_states
        self.state_k = _c(sys.state_k, np.int32)
        self.eps = _c(sys.eps, np.float64)
        self.kgrid = _c(sys.kgrid, np.int32)
        self.qgrid = _c(sys.qgrid, np.int32)
        self.nm = int(sys.n_modes)
        self.hw = _c(sys.hw, np.float64)
        self.nph = _c(nph, np.float64)
        assert self.hw.shape == self.nph.shape
        self.sigma = float(sys.sigma)
        self.nq = float(sys.n_q_norm)
        self.ci = _c(sys.ch_i, np.int32)
        self.cj = _c(sys.ch_j, np.int32)
        self.cn = _c(sys.ch_nu, np.int8)
        self.g2 = _c(sys.g2 if g2 is None else g2, np.float64)

    def common(self):
        return [self.S, _ptr(self.state_k), _ptr(self.eps), _ptr(self.kgrid), _ptr(self.qgrid),
                self.nm, _ptr(self.hw), _ptr(self.nph), self.sigma, self.nq,
                int(self.ci.size), _ptr(self.ci), _ptr(self.cj), _ptr(self.cn), _ptr(self.g2)]


# ---------------------------------------------------------------------------
# channel selection (scattering-channel paragraph after Eq. 2)
# ---------------------------------------------------------------------------
def channel_phonon_energy(sys):
    """hw(q, nu) of every channel, with q = k_j - k_i folded onto the q grid
    (the k grid is an integer multiple of the q grid along each axis)."""
    kg = np.asarray(sys.kgrid, np.int64)
    qg = np.asarray(sys.qgrid, np.int64)
    k = np.asarray(sys.state_k, np.int64)
    kc = np.stack([k // (kg[1] * kg[2]), (k // kg[2]) % kg[1], k % kg[2]], axis=1)
    dk = (kc[np.asarray(sys.ch_j)] - kc[np.asarray(sys.ch_i)]) % kg
    ratio = kg // qg
    assert np.all(dk % ratio == 0), "k_j - k_i must be a q-grid vector"
    q = dk // ratio
    qlin = (q[:, 0] * qg[1] + q[:, 1]) * qg[2] + q[:, 2]
    return np.asarray(sys.hw, np.float64)[qlin, np.asarray(sys.ch_nu, np.int64)]


def select_channels(sys, energy_nsigma=0.0, g2_min=0.0):
    """Keep mask [n_channels] of the channel selection.  A channel survives
    approximate energy conservation when one of its two Gaussian deltas, of
    eps_i - eps_j + hw (absorption) or eps_i - eps_j - hw (emission), lies
    within energy_nsigma standard deviations of its centre (0 disables the
    energy cut), and the |g|^2 cut when |g|^2 >= g2_min.  The comparison is
    taken in FP64, as the library takes it."""
    eps = np.asarray(sys.eps, np.float64)
    g2 = np.asarray(sys.g2, np.float64)
    keep = g2 >= float(g2_min)
    if energy_nsigma:
        d = eps[np.asarray(sys.ch_i)] - eps[np.asarray(sys.ch_j)]
        w = channel_phonon_energy(sys)
        keep &= np.minimum(np.abs(d + w), np.abs(d - w)) < float(energy_nsigma) * float(sys.sigma)
    return keep


def subset(sys, keep):
    """Copy of a system holding only the channels where keep is True."""
    import copy
    r = copy.copy(sys)
    for name in ("ch_i", "ch_j", "ch_nu", "g2"):
        setattr(r, name, np.asarray(getattr(sys, name))[keep])
    return r


# ---------------------------------------------------------------------------
# collision integral (Eq. 2)
# ---------------------------------------------------------------------------
def collision(sys, f, nph, g2=None, mask=None, args=None):
    """I[f] [S] in FP64 by the sequential channel-list loop.  mask (bool [S])
    restricts the accumulation to sampled destinations."""
    a = args or _Args(sys, nph, g2)
    f = _c(f, np.float64)
    I = np.zeros(a.S)
    m = None if mask is None else _c(mask, np.uint8)
    _lib().orc_collision(*a.common(), _ptr(f), _ptr(m), _ptr(I))
    return I


def _threaded(fname, a, f, n_out, threads, pass_mask):
    """Runs the C function fname over `threads` disjoint contiguous slices of
    the channel list at once (each ctypes call releases the GIL) and adds the
    slices' n_out partial [S] vectors in slice order."""
    from concurrent.futures import ThreadPoolExecutor
    n = int(a.ci.size)
    if threads is None:
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(int(threads), max(n, 1)))
    cuts = [n * t // threads for t in range(threads + 1)]
    parts = [[np.zeros(a.S) for _ in range(n_out)] for _ in range(threads)]
    base = a.common()
    fn = getattr(_lib(), fname)

    def run(t):
        b, e = cuts[t], cuts[t + 1]
        args_t = list(base)
        args_t[10] = e - b
        args_t[11] = ctypes.c_void_p(a.ci.ctypes.data + 4 * b)
        args_t[12] = ctypes.c_void_p(a.cj.ctypes.data + 4 * b)
        args_t[13] = ctypes.c_void_p(a.cn.ctypes.data + b)
        args_t[14] = ctypes.c_void_p(a.g2.ctypes.data + 8 * b)
        extra = [None] if pass_mask else []
        fn(*args_t, _ptr(f), *extra, *[_ptr(x) for x in parts[t]])

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, range(threads)))
    out = [np.zeros(a.S) for _ in range(n_out)]
    for pt in parts:
        for k in range(n_out):
            out[k] += pt[k]
    return out


def collision_threads(sys, f, nph, threads=None, g2=None, args=None):
    """I[f] [S] by the same sequential C channel loop as collision(), run on
    `threads` disjoint contiguous slices of the channel list at once; the
    slices' partial vectors are added in slice order.  The result equals
    collision() up to the order of the floating-point additions.
    threads=None uses every CPU of the process."""
    a = args or _Args(sys, nph, g2)
    return _threaded("orc_collision", a, _c(f, np.float64), 1, threads, True)[0]


def collision_inout_threads(sys, f, nph, threads=None, g2=None, args=None):
    """(in-scattering, out-scattering) [S] as collision_inout(), on threads
    like collision_threads()."""
    a = args or _Args(sys, nph, g2)
    rin, rout = _threaded("orc_collision_inout", a, _c(f, np.float64), 2, threads, False)
    return rin, rout


def collision_inout(sys, f, nph, g2=None):
    """(in-scattering, out-scattering) rates [S]; I = in - out."""
    a = _Args(sys, nph, g2)
    f = _c(f, np.float64)
    rin, rout = np.zeros(a.S), np.zeros(a.S)
    _lib().orc_collision_inout(*a.common(), _ptr(f), _ptr(rin), _ptr(rout))
    return rin, rout


def collision_batched(sys, F, nph, g2=None):
    """Columns of I for a batch F [B, S]: the plain oracle applied per vector."""
    a = _Args(sys, nph, g2)
    return np.stack([collision(sys, F[b], nph, args=a) for b in range(F.shape[0])])


def collision_vjp(sys, f, nph, lam, g2=None, want_f=True, want_g2=True):
    """(dL/df [S], dL/dg2 [Nch]) for L = sum_d lam_d I_d."""
    a = _Args(sys, nph, g2)
    f = _c(f, np.float64)
    lam = _c(lam, np.float64)
    gf = np.zeros(a.S) if want_f else None
    gg = np.zeros(a.ci.size) if want_g2 else None
    _lib().orc_collision_vjp(*a.common(), _ptr(f), _ptr(lam), _ptr(gf), _ptr(gg))
    return gf, gg


def collision_elastic(sys, f, modes=None, g2=None):
    """Elastic collision integral [S] in FP64 over the channels whose mode is
    in modes (all when None).  A static perturbation (a defect) moves an
    electron between states of equal energy with no phonon: by Fermi's golden
    rule the rate is C |g|^2 G(e_i - e_j) with C = 2 pi / (hbar N_q) and G the
    normalised Gaussian of width sigma, and the Pauli factors leave f_j - f_i.
    Each channel adds its term to I_i and subtracts it from I_j."""
    ci = np.asarray(sys.ch_i, np.int64)
    cj = np.asarray(sys.ch_j, np.int64)
    g = np.asarray(sys.g2 if g2 is None else g2, np.float64)
    if modes is not None:
        sel = np.isin(np.asarray(sys.ch_nu), np.asarray(modes))
        ci, cj, g = ci[sel], cj[sel], g[sel]
    eps = np.asarray(sys.eps, np.float64)
    f = np.asarray(f, np.float64)
    sig = float(sys.sigma)
    d = eps[ci] - eps[cj]
    G = np.exp(-0.5 * (d / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    X = 2.0 * np.pi / (HBAR_EV_FS * float(sys.n_q_norm)) * g * G * (f[cj] - f[ci])
    I = np.zeros(int(sys.n_states))
    np.add.at(I, ci, X)
    np.add.at(I, cj, -X)
    return I


def _bose_terms(sys, n, nph, g2):
    """Per orientation (destination d, partner p) of every channel: the arrays
    the Bose collision integral and its reverse mode are built from."""
    ci, cj, nu, qij, qji = _channel_geometry(sys)
    hw = np.asarray(sys.hw, np.float64)
    N = np.asarray(nph, np.float64)
    eps = np.asarray(sys.eps, np.float64)
    g = np.asarray(sys.g2 if g2 is None else g2, np.float64)
    sig = float(sys.sigma)
    G = lambda x: np.exp(-0.5 * (x / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    C = 2.0 * np.pi / HBAR_EV_FS / float(sys.n_q_norm)
    out = []
    for d, p, q in ((ci, cj, qij), (cj, ci, qji)):
        w, Nq = hw[q, nu], N[q, nu]
        x = eps[d] - eps[p]
        Gp, Gm = G(x + w), G(x - w)
        out.append((d, p, q, Gp, Gm, Nq))
    return out, g, C


def collision_bose(sys, n, nph, g2=None):
    """Phonon-phonon (three-phonon) collision integral [S] in FP64 over the
    channel list (Discussion: other scattering mechanisms on the same data
    structure).  The states are phonon modes with energies e = eps and
    occupations n; a channel (i, j, nu) couples modes d and p through the
    third phonon (nu, q = q_p - q_d, energy w, occupation N), and the golden
    rule of Eq. 2 applies with Bose factors: a mode that receives a quantum
    carries the enhancement 1 + n where a fermion carries 1 - f.  For
    x = e_d - e_p the four processes give mode d
      G(x - w) [n_p N (1 + n_d) - n_d (1 + n_p)(N + 1)]   (p + phonon <-> d)
      G(x + w) [n_p (1 + n_d)(N + 1) - n_d N (1 + n_p)]   (p <-> d + phonon)
    times C |V|^2, C = 2 pi / (hbar N_q), summed over both orientations of
    every channel."""
    n = np.asarray(n, np.float64)
    terms, g, C = _bose_terms(sys, n, nph, g2)
    I = np.zeros(int(sys.n_states))
    for d, p, q, Gp, Gm, Nq in terms:
        gain = n[p] * (1.0 + n[d])
        loss = n[d] * (1.0 + n[p])
        T = C * g * (Gm * (gain * Nq - loss * (Nq + 1.0)) + Gp * (gain * (Nq + 1.0) - loss * Nq))
        np.add.at(I, d, T)
    return I


def collision_bose_vjp(sys, n, nph, lam, g2=None):
    """(dL/dn [S], dL/dg2 [n_channels], dL/dN [Nq, n_modes]) for
    L = sum_d lam_d I_d of collision_bose.  Per orientation the term is
    C |V|^2 (A gain - B loss) with A = G(x - w) N + G(x + w)(N + 1),
    B = G(x - w)(N + 1) + G(x + w) N, gain = n_p (1 + n_d), loss = n_d (1 + n_p);
    its derivatives: d/dn_d = C |V|^2 (A n_p - B (1 + n_p)),
    d/dn_p = C |V|^2 (A (1 + n_d) - B n_d), d/d|V|^2 = C (A gain - B loss),
    d/dN = C |V|^2 (G(x - w) + G(x + w)) (gain - loss)."""
    n = np.asarray(n, np.float64)
    lam = np.asarray(lam, np.float64)
    terms, g, C = _bose_terms(sys, n, nph, g2)
    nm = int(sys.n_modes)
    nu = np.asarray(sys.ch_nu, np.int64)
    gn = np.zeros(int(sys.n_states))
    gg = np.zeros(g.size)
    gN = np.zeros(np.asarray(sys.hw).size)
    for d, p, q, Gp, Gm, Nq in terms:
        A = Gm * Nq + Gp * (Nq + 1.0)
        B = Gm * (Nq + 1.0) + Gp * Nq
        gain = n[p] * (1.0 + n[d])
        loss = n[d] * (1.0 + n[p])
        l = lam[d]
        np.add.at(gn, d, l * C * g * (A * n[p] - B * (1.0 + n[p])))
        np.add.at(gn, p, l * C * g * (A * (1.0 + n[d]) - B * n[d]))
        gg += l * C * (A * gain - B * loss)
        np.add.at(gN, q * nm + nu, l * C * g * (Gm + Gp) * (gain - loss))
    return gn, gg, gN.reshape(np.asarray(sys.hw).shape)


def collision_brute(sys, f, nph):
    """Eq. 2 literally: for every state (n,k), sum over every q of the q grid,
    every band m and mode nu, with the partner (m, k+q) looked up on the k grid.
    |g|^2 comes from the channel list (0 for inactive channels); terms with
    hw < 1e-6 eV have no active channel.  Tiny grids only (dense [S,S,modes])."""
    S, nm = sys.n_states, sys.n_modes
    kg = np.asarray(sys.kgrid)
    qg = np.asarray(sys.qgrid)
    r = kg // qg
    g2d = np.zeros((S, S, nm))
    np.add.at(g2d, (sys.ch_i, sys.ch_j, sys.ch_nu.astype(np.int64)), sys.g2)
    np.add.at(g2d, (sys.ch_j, sys.ch_i, sys.ch_nu.astype(np.int64)), sys.g2)
    nk = int(np.prod(kg))
    kc = np.stack(np.unravel_index(sys.state_k, tuple(kg)), axis=1)
    at_k = [[] for _ in range(nk)]
    for s, k in enumerate(sys.state_k):
        at_k[int(k)].append(s)
    qc = np.stack(np.unravel_index(np.arange(int(np.prod(qg))), tuple(qg)), axis=1)
    pref = 2.0 * np.pi / HBAR_EV_FS / sys.n_q_norm
    sig = sys.sigma
    G = lambda x: np.exp(-0.5 * (x / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    I = np.zeros(S)
    for d in range(S):
        kp = (kc[d][None, :] + r[None, :] * qc) % kg[None, :]
        kp_lin = np.ravel_multi_index(tuple(kp.T), tuple(kg))
        total = 0.0
        for qi in range(qc.shape[0]):
            for p in at_k[int(kp_lin[qi])]:
                for nu in range(nm):
                    g = g2d[d, p, nu]
                    if g == 0.0:
                        continue
                    w = sys.hw[qi, nu]
                    N = nph[qi, nu]
                    fd, fp = f[d], f[p]
                    F_abs = fd * (1 - fp) * N - fp * (1 - fd) * (N + 1)
                    F_em = fd * (1 - fp) * (N + 1) - fp * (1 - fd) * N
                    de = sys.eps[d] - sys.eps[p]
                    total += -pref * g * (G(de + w) * F_abs + G(de - w) * F_em)
        I[d] = total
    return I


# ---------------------------------------------------------------------------
# phonon side of the same processes (coupled electron-phonon dynamics)
# ---------------------------------------------------------------------------
def phonon_rate(sys, f, nph, g2=None):
    """dN/dt [Nq, n_modes] from electron-phonon processes over the channel list.

    A channel (i, j, nu) with q = k_j - k_i (on the q grid) carries four
    golden-rule processes: i -> j absorbing (nu, q) and its reverse j -> i
    emitting (nu, q), both with the delta G(e_i - e_j + hw); and i -> j
    emitting (nu, -q) with its reverse absorbing (nu, -q), both with
    G(e_i - e_j - hw).  Phonon (nu, q) gains the emissions and loses the
    absorptions:
      dN(nu, q)  += Cp |g|^2 G(e_i - e_j + hw) [(N+1) f_j (1 - f_i) - N f_i (1 - f_j)]
      dN(nu, -q) += Cp |g|^2 G(e_i - e_j - hw) [(N+1) f_i (1 - f_j) - N f_j (1 - f_i)]
    with N and hw of the bin (tables even in q), Cp = 2 pi / (hbar N_k) and
    N_k the full k-grid count (the electron side carries 1 / N_q)."""
    kg = np.asarray(sys.kgrid, np.int64)
    qg = np.asarray(sys.qgrid, np.int64)
    nm = int(sys.n_modes)
    k = np.asarray(sys.state_k, np.int64)
    kc = np.stack([k // (kg[1] * kg[2]), (k // kg[2]) % kg[1], k % kg[2]], axis=1)
    ci = np.asarray(sys.ch_i, np.int64)
    cj = np.asarray(sys.ch_j, np.int64)
    nu = np.asarray(sys.ch_nu, np.int64)
    g = np.asarray(sys.g2 if g2 is None else g2, np.float64)
    ratio = kg // qg

    def qlin(dk):
        q = (dk % kg) // ratio
        return (q[:, 0] * qg[1] + q[:, 1]) * qg[2] + q[:, 2]

    qp = qlin(kc[cj] - kc[ci])          # q = k_j - k_i
    qm = qlin(kc[ci] - kc[cj])          # -q
    hw = np.asarray(sys.hw, np.float64)
    N = np.asarray(nph, np.float64)
    eps = np.asarray(sys.eps, np.float64)
    f = np.asarray(f, np.float64)
    sig = float(sys.sigma)
    G = lambda x: np.exp(-0.5 * (x / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    Cp = 2.0 * np.pi / (HBAR_EV_FS * float(np.prod(kg)))
    d = eps[ci] - eps[cj]
    w1, n1 = hw[qp, nu], N[qp, nu]
    w2, n2 = hw[qm, nu], N[qm, nu]
    y1 = Cp * g * G(d + w1) * ((n1 + 1) * f[cj] * (1 - f[ci]) - n1 * f[ci] * (1 - f[cj]))
    y2 = Cp * g * G(d - w2) * ((n2 + 1) * f[ci] * (1 - f[cj]) - n2 * f[cj] * (1 - f[ci]))
    out = np.zeros(hw.size)
    np.add.at(out, qp * nm + nu, y1)
    np.add.at(out, qm * nm + nu, y2)
    return out.reshape(hw.shape)


def _channel_geometry(sys):
    """(ci, cj, nu, q_ij, q_ji) of the channel list: q_ij = k_j - k_i and
    q_ji = k_i - k_j as linear q-grid indices (numpy, independent of the C
    code)."""
    kg = np.asarray(sys.kgrid, np.int64)
    qg = np.asarray(sys.qgrid, np.int64)
    k = np.asarray(sys.state_k, np.int64)
    kc = np.stack([k // (kg[1] * kg[2]), (k // kg[2]) % kg[1], k % kg[2]], axis=1)
    ci = np.asarray(sys.ch_i, np.int64)
    cj = np.asarray(sys.ch_j, np.int64)
    ratio = kg // qg

    def qlin(dk):
        q = (dk % kg) // ratio
        return (q[:, 0] * qg[1] + q[:, 1]) * qg[2] + q[:, 2]

    return ci, cj, np.asarray(sys.ch_nu, np.int64), qlin(kc[cj] - kc[ci]), qlin(kc[ci] - kc[cj])


def collision_vjp_nph(sys, f, nph, lam, g2=None):
    """dL/dN [Nq, n_modes] for L = sum_d lam_d I_d.  In Eq. 2 the occupation
    factors are affine in N: dF_abs/dN = dF_em/dN = f_d - f_p, so the summand
    of destination d and partner p through (nu, q = k_p - k_d) has
    dT/dN(nu, q) = -(2 pi / hbar)(1/N_q) |g|^2 [G(e_d - e_p + hw) + G(e_d - e_p - hw)] (f_d - f_p).
    Each channel contributes from both of its orientations, each at its own q."""
    ci, cj, nu, qij, qji = _channel_geometry(sys)
    hw = np.asarray(sys.hw, np.float64)
    eps = np.asarray(sys.eps, np.float64)
    f = np.asarray(f, np.float64)
    lam = np.asarray(lam, np.float64)
    g = np.asarray(sys.g2 if g2 is None else g2, np.float64)
    sig = float(sys.sigma)
    G = lambda x: np.exp(-0.5 * (x / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    P = 2.0 * np.pi / HBAR_EV_FS / float(sys.n_q_norm)
    nm = int(sys.n_modes)
    out = np.zeros(hw.size)
    for d, p, q in ((ci, cj, qij), (cj, ci, qji)):
        w = hw[q, nu]
        de = eps[d] - eps[p]
        dT = -P * g * (G(de + w) + G(de - w)) * (f[d] - f[p])
        np.add.at(out, q * nm + nu, lam[d] * dT)
    return out.reshape(hw.shape)


def phonon_rate_vjp(sys, f, nph, mu, g2=None):
    """(dL/df [S], dL/dN [Nq, n_modes], dL/dg2 [n_channels]) for
    L = sum_{q, nu} mu(q, nu) dN/dt(q, nu), from the two terms per channel of
    phonon_rate (q = k_j - k_i):
      y1 = Cp |g|^2 G(e_i - e_j + hw(q)) [(N(q)+1) f_j (1-f_i) - N(q) f_i (1-f_j)]    -> bin q
      y2 = Cp |g|^2 G(e_i - e_j - hw(-q)) [(N(-q)+1) f_i (1-f_j) - N(-q) f_j (1-f_i)] -> bin -q
    differentiated by hand:
      dy1/df_i = -Cp |g|^2 Ga (N(q) + f_j),      dy1/df_j = Cp |g|^2 Ga (N(q) + 1 - f_i),
      dy2/df_i =  Cp |g|^2 Ge (N(-q) + 1 - f_j), dy2/df_j = -Cp |g|^2 Ge (N(-q) + f_i),
      dy1/dN(q) = Cp |g|^2 Ga (f_j - f_i),       dy2/dN(-q) = Cp |g|^2 Ge (f_i - f_j),
      dy/d|g|^2 = y / |g|^2."""
    ci, cj, nu, qp, qm = _channel_geometry(sys)
    hw = np.asarray(sys.hw, np.float64)
    N = np.asarray(nph, np.float64)
    eps = np.asarray(sys.eps, np.float64)
    f = np.asarray(f, np.float64)
    mu = np.asarray(mu, np.float64)
    g = np.asarray(sys.g2 if g2 is None else g2, np.float64)
    sig = float(sys.sigma)
    G = lambda x: np.exp(-0.5 * (x / sig) ** 2) / (sig * np.sqrt(2.0 * np.pi))
    Cp = 2.0 * np.pi / (HBAR_EV_FS * float(np.prod(np.asarray(sys.kgrid, np.int64))))
    d = eps[ci] - eps[cj]
    n1, n2 = N[qp, nu], N[qm, nu]
    m1, m2 = mu[qp, nu], mu[qm, nu]
    Ga = G(d + hw[qp, nu])
    Ge = G(d - hw[qm, nu])
    fi, fj = f[ci], f[cj]
    gf = np.zeros(f.size)
    np.add.at(gf, ci, Cp * g * (-m1 * Ga * (n1 + fj) + m2 * Ge * (n2 + 1.0 - fj)))
    np.add.at(gf, cj, Cp * g * (m1 * Ga * (n1 + 1.0 - fi) - m2 * Ge * (n2 + fi)))
    gN = np.zeros(hw.size)
    nm = int(sys.n_modes)
    np.add.at(gN, qp * nm + nu, m1 * Cp * g * Ga * (fj - fi))
    np.add.at(gN, qm * nm + nu, m2 * Cp * g * Ge * (fi - fj))
    gg = Cp * (m1 * Ga * ((n1 + 1.0) * fj * (1.0 - fi) - n1 * fi * (1.0 - fj))
               + m2 * Ge * ((n2 + 1.0) * fi * (1.0 - fj) - n2 * fj * (1.0 - fi)))
    return gf, gN.reshape(hw.shape), gg


def rk4_coupled_adjoint_step(sys, stages, dt, gbar_f, gbar_N, g2=None):
    """Reverse of one rk4_coupled_step.  stages = ((u1, M1), .., (u4, M4)), the
    stage inputs of the step; (gbar_f, gbar_N) = dL/d(f, N) after the step.
    The right-hand side is F(u, M) = (I(u, M), E R(u, M)) with E the even part
    in q (a symmetric averaging, E^T = E), so its transposed Jacobian maps
    (a, b) to (J_If^T a + J_Rf^T E b, J_IN^T a + J_RN^T E b), and the |g|^2
    gradient to J_Ig^T a + J_Rg^T E b.  Returns (dL/df, dL/dN, dL/dg2 of the step)."""

    def vjp(u, M, a, b):
        gf_I, gg_I = collision_vjp(sys, u, M, a, g2=g2)
        gN_I = collision_vjp_nph(sys, u, M, a, g2=g2)
        gf_R, gN_R, gg_R = phonon_rate_vjp(sys, u, M, even_in_q(sys, b), g2=g2)
        return gf_I + gf_R, gN_I + gN_R, gg_I + gg_R

    gbar_f = np.asarray(gbar_f, np.float64)
    gbar_N = np.asarray(gbar_N, np.float64)
    (u1, M1), (u2, M2), (u3, M3), (u4, M4) = stages
    a4, b4 = (dt / 6.0) * gbar_f, (dt / 6.0) * gbar_N
    uf4, uN4, gg4 = vjp(u4, M4, a4, b4)
    a3, b3 = (dt / 3.0) * gbar_f + dt * uf4, (dt / 3.0) * gbar_N + dt * uN4
    uf3, uN3, gg3 = vjp(u3, M3, a3, b3)
    a2, b2 = (dt / 3.0) * gbar_f + 0.5 * dt * uf3, (dt / 3.0) * gbar_N + 0.5 * dt * uN3
    uf2, uN2, gg2_ = vjp(u2, M2, a2, b2)
    a1, b1 = (dt / 6.0) * gbar_f + 0.5 * dt * uf2, (dt / 6.0) * gbar_N + 0.5 * dt * uN2
    uf1, uN1, gg1 = vjp(u1, M1, a1, b1)
    return (gbar_f + uf1 + uf2 + uf3 + uf4, gbar_N + uN1 + uN2 + uN3 + uN4,
            gg1 + gg2_ + gg3 + gg4)


def rk4_coupled_trajectory_grad(sys, f0, N0, dt, n_steps, gfT, gNT, g2=None):
    """Gradients of L(f_T, N_T) through n_steps coupled RK4 steps, storing
    every stage: returns (f_T, N_T, dL/df0, dL/dN0, dL/dg2)."""
    f = np.array(f0, dtype=np.float64)
    N = np.array(N0, dtype=np.float64)
    steps = []
    for _ in range(n_steps):
        f, N, st = _rk4_coupled_with_stages(sys, f, N, dt, g2)
        steps.append(st)
    gf = np.array(gfT, dtype=np.float64)
    gN = np.array(gNT, dtype=np.float64)
    gg = np.zeros(sys.n_channels)
    for st in reversed(steps):
        gf, gN, dg = rk4_coupled_adjoint_step(sys, st, dt, gf, gN, g2=g2)
        gg += dg
    return f, N, gf, gN, gg


def _rk4_coupled_with_stages(sys, f, nph, dt, g2):
    """rk4_coupled_step that also returns its stage inputs."""

    def rhs(u, M):
        return collision(sys, u, M, g2=g2), even_in_q(sys, phonon_rate(sys, u, M, g2=g2))
    u1, M1 = np.array(f, dtype=np.float64), np.array(nph, dtype=np.float64)
    k1, p1 = rhs(u1, M1)
    u2, M2 = u1 + 0.5 * dt * k1, M1 + 0.5 * dt * p1
    k2, p2 = rhs(u2, M2)
    u3, M3 = u1 + 0.5 * dt * k2, M1 + 0.5 * dt * p2
    k3, p3 = rhs(u3, M3)
    u4, M4 = u1 + dt * k3, M1 + dt * p3
    k4, p4 = rhs(u4, M4)
    return (u1 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4),
            M1 + (dt / 6.0) * (p1 + 2.0 * p2 + 2.0 * p3 + p4),
            ((u1, M1), (u2, M2), (u3, M3), (u4, M4)))


# ---------------------------------------------------------------------------
# field term of Eq. 1 (drift in k space)
# ---------------------------------------------------------------------------
def drift_neighbors(sys):
    """[S, 3, 2] index of the state of the same band one k-grid step above
    (column 0) and below (column 1) along each axis, periodic over the grid;
    -1 when that state is not in the list (outside the energy window)."""
    kg = np.asarray(sys.kgrid, np.int64)
    k = np.asarray(sys.state_k, np.int64)
    band = np.asarray(sys.state_band, np.int64)
    c = np.stack([k // (kg[1] * kg[2]), (k // kg[2]) % kg[1], k % kg[2]], axis=1)
    where = {}
    for s in range(k.size):
        key = (int(k[s]), int(band[s]))
        assert key not in where, "two states share (k, band)"
        where[key] = s
    nbr = np.full((k.size, 3, 2), -1, np.int64)
    for s in range(k.size):
        for a in range(3):
            for col, step in ((0, 1), (1, -1)):
                cc = c[s].copy()
                cc[a] = (cc[a] + step) % kg[a]
                kk = int((cc[0] * kg[1] + cc[1]) * kg[2] + cc[2])
                nbr[s, a, col] = where.get((kk, int(band[s])), -1)
    return nbr


def drift(sys, f, rates, nbr=None):
    """Field term of Eq. 1, -(1/hbar) F . grad_k f, with the derivative along
    axis a taken as the central difference (f(k + dk_a) - f(k - dk_a)) /
    (2 dk_a) inside the state's band: D_s = -sum_a r_a (f_up - f_down) / 2,
    r_a = F_a / (hbar dk_a) in 1/fs.  A neighbour outside the list has f = 0."""
    nbr = drift_neighbors(sys) if nbr is None else nbr
    f = np.asarray(f, np.float64)
    fx = np.concatenate([f, [0.0]])          # index -1 reads the appended 0
    D = np.zeros(f.size)
    for a in range(3):
        D -= float(rates[a]) * 0.5 * (fx[nbr[:, a, 0]] - fx[nbr[:, a, 1]])
    return D


def drift_transpose(sys, lam, rates, nbr=None):
    """D^T lam, by scattering each row of D: row s has -r_a/2 in the column of
    its upper neighbour and +r_a/2 in the column of its lower one."""
    nbr = drift_neighbors(sys) if nbr is None else nbr
    lam = np.asarray(lam, np.float64)
    out = np.zeros(lam.size + 1)             # slot -1 collects missing neighbours
    for a in range(3):
        np.add.at(out, nbr[:, a, 0], -0.5 * float(rates[a]) * lam)
        np.add.at(out, nbr[:, a, 1], 0.5 * float(rates[a]) * lam)
    return out[:-1]


# ---------------------------------------------------------------------------
# real-time BTE: classical RK4 and its discrete adjoint
# ---------------------------------------------------------------------------
def rk4_step(sys, f, nph, dt, g2=None, return_stages=False, rates=None, nbr=None, statistics="fermi"):
    """One classical fourth-order Runge-Kutta step of df/dt = I[f] (+ the
    drift term of Eq. 1 when rates is given).  statistics="bose": dn/dt of
    collision_bose (phonon modes as the states; no drift term)."""
    a = _Args(sys, nph, g2)
    if statistics == "bose":
        assert rates is None
        I = lambda u: collision_bose(sys, u, nph, g2=g2)
    elif rates is None:
        I = lambda u: collision(sys, u, nph, args=a)
    else:
        nbr = drift_neighbors(sys) if nbr is None else nbr
        I = lambda u: collision(sys, u, nph, args=a) + drift(sys, u, rates, nbr)
    u1 = np.array(f, dtype=np.float64)
    k1 = I(u1)
    u2 = u1 + 0.5 * dt * k1
    k2 = I(u2)
    u3 = u1 + 0.5 * dt * k2
    k3 = I(u3)
    u4 = u1 + dt * k3
    k4 = I(u4)
    out = u1 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return (out, (u1, u2, u3, u4)) if return_stages else out


def even_in_q(sys, x):
    """(x(q) + x(-q)) / 2 of a [Nq, n_modes] table."""
    qg = np.asarray(sys.qgrid, np.int64)
    q = np.arange(int(np.prod(qg)))
    c = np.stack([q // (qg[1] * qg[2]), (q // qg[2]) % qg[1], q % qg[2]], axis=1)
    m = (-c) % qg
    qm = (m[:, 0] * qg[1] + m[:, 1]) * qg[2] + m[:, 2]
    x = np.asarray(x, np.float64)
    return 0.5 * (x + x[qm])


def rk4_coupled_step(sys, f, nph, dt, g2=None):
    """One classical RK4 step of the coupled system df/dt = I[f, N],
    dN/dt = even part in q of phonon_rate(f, N): electrons and phonons
    advanced together.  Eq. 2 evaluates each orientation of a channel with N
    at its own q, which is exact for N even in q; the phonons of q and -q are
    therefore evolved as a pair (the even part of the rate), which keeps N even
    and, with hw even, leaves every energy transfer unchanged."""

    def rhs(u, M):
        return collision(sys, u, M, g2=g2), even_in_q(sys, phonon_rate(sys, u, M, g2=g2))
    u1, M1 = np.array(f, dtype=np.float64), np.array(nph, dtype=np.float64)
    k1, p1 = rhs(u1, M1)
    u2, M2 = u1 + 0.5 * dt * k1, M1 + 0.5 * dt * p1
    k2, p2 = rhs(u2, M2)
    u3, M3 = u1 + 0.5 * dt * k2, M1 + 0.5 * dt * p2
    k3, p3 = rhs(u3, M3)
    u4, M4 = u1 + dt * k3, M1 + dt * p3
    k4, p4 = rhs(u4, M4)
    return (u1 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4),
            M1 + (dt / 6.0) * (p1 + 2.0 * p2 + 2.0 * p3 + p4))


def rk4_adjoint_step(sys, stages, nph, dt, gbar, g2=None, rates=None, nbr=None, statistics="fermi"):
    """Reverse of one RK4 step.  Given gbar = dL/df_{n+1} and the stage inputs
    (u1..u4) of the step, return (dL/df_n, dL/dg2 contribution of the step).
    With rates, each stage's transposed Jacobian also holds D^T."""
    u1, u2, u3, u4 = stages
    if statistics == "bose":
        assert rates is None
        vjp = lambda u, lam: collision_bose_vjp(sys, u, nph, lam, g2=g2)[:2]
    elif rates is None:
        vjp = lambda u, lam: collision_vjp(sys, u, nph, lam, g2=g2)
    else:
        nbr = drift_neighbors(sys) if nbr is None else nbr

        def vjp(u, lam):
            gf, gg = collision_vjp(sys, u, nph, lam, g2=g2)
            return gf + drift_transpose(sys, lam, rates, nbr), gg
    kb4 = (dt / 6.0) * gbar
    ub4, gg4 = vjp(u4, kb4)
    kb3 = (dt / 3.0) * gbar + dt * ub4
    ub3, gg3 = vjp(u3, kb3)
    kb2 = (dt / 3.0) * gbar + 0.5 * dt * ub3
    ub2, gg2_ = vjp(u2, kb2)
    kb1 = (dt / 6.0) * gbar + 0.5 * dt * ub2
    ub1, gg1 = vjp(u1, kb1)
    return gbar + ub1 + ub2 + ub3 + ub4, gg1 + gg2_ + gg3 + gg4


def rk4_trajectory_grad(sys, f0, nph, dt, n_steps, gT, g2=None, rates=None, statistics="fermi"):
    """Gradients of L(f_T) through n_steps RK4 steps, storing every stage."""
    nbr = None if rates is None else drift_neighbors(sys)
    f = np.array(f0, dtype=np.float64)
    stages = []
    for _ in range(n_steps):
        f, st = rk4_step(sys, f, nph, dt, g2=g2, return_stages=True, rates=rates, nbr=nbr, statistics=statistics)
        stages.append(st)
    g = np.array(gT, dtype=np.float64)
    gg = np.zeros(sys.n_channels)
    for st in reversed(stages):
        g, dg = rk4_adjoint_step(sys, st, nph, dt, g, g2=g2, rates=rates, nbr=nbr, statistics=statistics)
        gg += dg
    return f, g, gg


# ---------------------------------------------------------------------------
# transport: linearised steady-state BTE
# ---------------------------------------------------------------------------
def transport_coeffs(sys, f0, nph, g2=None):
    """(tau_inv [S], W_ij [Nch], W_ji [Nch]): dI/df at f0 split into its
    diagonal (-tau_inv) and the off-diagonal entries of each channel."""
    a = _Args(sys, nph, g2)
    f0 = _c(f0, np.float64)
    tau_inv = np.zeros(a.S)
    Wij = np.zeros(a.ci.size)
    Wji = np.zeros(a.ci.size)
    _lib().orc_transport_coeffs(*a.common(), _ptr(f0), _ptr(tau_inv), _ptr(Wij), _ptr(Wji))
    return tau_inv, Wij, Wji


def dfde_fd(f0, T):
    """d f0 / d eps of a Fermi-Dirac distribution at temperature T, from f0."""
    return -np.asarray(f0) * (1.0 - np.asarray(f0)) / (KB_EV_K * T)


def mobility_cm2(vel, x, f0):
    """mu_ab = -e sum_d v_a x_b / sum_d f0 with x in fs*(m/s)/eV and v in m/s
    (e = 1 in eV units): 1 fs = 1e-15 s and 1 m^2 = 1e4 cm^2."""
    return -1e-15 * 1e4 * (np.asarray(vel).T @ np.asarray(x)) / float(np.sum(f0))


def transport_apply_W(sys, Wij, Wji, x):
    """(W x)_d = sum over channels of the off-diagonal rows, for x [S, 3]."""
    S = sys.n_states
    out = np.zeros_like(x)
    for b in range(x.shape[1]):
        out[:, b] = (np.bincount(sys.ch_i, weights=Wij * x[sys.ch_j, b], minlength=S)
                     + np.bincount(sys.ch_j, weights=Wji * x[sys.ch_i, b], minlength=S))
    return out


def transport_solve(sys, f0, vel, T, nph, tol=1e-8, max_iter=200, g2=None, stop_on_tol=True,
                    stall=5):
    """Iterate x_d = tau_d (v_d df0/de + sum_p W_dp x_p) from the RTA start
    until the mobility changes by at most tol (relative, max norm), or until
    that change has not fallen below its smallest value for `stall`
    iterations (the floor of the working precision; stagnated=True).
    Returns dict(mu [3,3] cm^2/Vs, x [S,3], iters, converged, stagnated,
    history, resid)."""
    tau_inv, Wij, Wji = transport_coeffs(sys, f0, nph, g2)
    # a state without any scattering (tau_inv = 0) is left out: x_d = 0
    tau = np.where(tau_inv > 0, 1.0 / np.where(tau_inv > 0, tau_inv, 1.0), 0.0)
    b = np.asarray(vel) * dfde_fd(f0, T)[:, None]
    x = tau[:, None] * b
    mu = mobility_cm2(vel, x, f0)
    hist = [mu]
    best, since = np.inf, 0
    for it in range(1, max_iter + 1):
        x = tau[:, None] * (b + transport_apply_W(sys, Wij, Wji, x))
        mu_new = mobility_cm2(vel, x, f0)
        rel = np.abs(mu_new - mu).max() / np.abs(mu_new).max()
        mu = mu_new
        hist.append(mu)
        if stop_on_tol and rel <= tol:
            return dict(mu=mu, x=x, iters=it, converged=True, stagnated=False, history=hist, resid=rel)
        if rel < best:
            best, since = rel, 0
        else:
            since += 1
        if stop_on_tol and since >= stall:
            return dict(mu=mu, x=x, iters=it, converged=False, stagnated=True, history=hist, resid=rel)
    return dict(mu=mu, x=x, iters=max_iter, converged=False, stagnated=False, history=hist, resid=rel)
