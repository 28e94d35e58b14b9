"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, validates problems before touching a device, and its host layout
builder (the destination-sorted target layer) has the documented invariants."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2511_03683_amd as E
import synth
from paper_2511_03683_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "ephbte.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ephbte_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = E.load_library()
    names = _declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SYMBOLS), "binding and header disagree"


def test_status_strings():
    assert E.status_string(0) == "ok"
    assert E.status_string(1) == "invalid argument"
    assert E.status_string(5) == "not converged"
    assert E.status_string(99) == "unknown status"


def test_null_plan_is_rejected():
    lib = E.load_library()
    st = lib.ephbte_collision_integral(None, 1, None, 1, None, 0, None, 1, None)
    assert st == binding.INVALID_ARGUMENT
    assert "plan" in E.last_error()
    assert lib.ephbte_plan_bytes(None) == 0
    lib.ephbte_destroy(None)


def _check_layout(s):
    rp, partner, mode, chan = E.layout_host(s)
    S, nch = s.n_states, s.n_channels
    assert rp[0] == 0 and rp[-1] == 2 * nch and np.all(np.diff(rp) >= 0)
    dest = np.repeat(np.arange(S), np.diff(rp))
    key = partner.astype(np.int64) * 8 + mode
    for d in range(S):
        seg = key[rp[d]:rp[d + 1]]
        assert np.all(np.diff(seg) > 0), "entries of a destination sorted by (partner, mode)"
    # each channel appears twice, once per endpoint, with the other endpoint as partner
    counts = np.bincount(chan, minlength=nch)
    assert np.all(counts == 2)
    ci, cj, cn = s.ch_i[chan], s.ch_j[chan], s.ch_nu[chan]
    assert np.all(mode == cn)
    assert np.all(((dest == ci) & (partner == cj)) | ((dest == cj) & (partner == ci)))
    assert np.all(partner != dest)
    return rp, partner, mode, chan


@pytest.mark.parametrize("maker", [lambda: synth.parabolic_system(4),
                                   lambda: synth.multiband_system(),
                                   lambda: synth.random_channel_system(n_states=50, n_channels=700),
                                   lambda: synth.ladder_system()])
def test_layout_invariants(maker):
    _check_layout(maker())


def test_layout_of_lexicographic_input_keeps_channel_order_for_primary_entries():
    s = synth.parabolic_system(4)
    rp, partner, mode, chan = _check_layout(s)
    dest = np.repeat(np.arange(s.n_states), np.diff(rp))
    prim = partner > dest
    assert np.all(np.diff(chan[prim]) == 1), "primary entries enumerate channels in order"


def test_layout_empty_and_isolated_states():
    s = synth.random_channel_system(n_states=20, n_channels=0)
    rp, partner, mode, chan = E.layout_host(s)
    assert rp.tolist() == [0] * 21
    s2 = synth.two_state_system()
    s2.eps = np.array([0.0, 0.05, 0.3])
    s2.state_k = np.array([0, 1, 1], np.int32)
    rp, *_ = E.layout_host(s2)
    assert rp.tolist() == [0, 1, 2, 2]


@pytest.mark.parametrize("nsig,g2min", [(2.5, 0.0), (1.0, 1e-3), (0.0, 1.5e-3), (40.0, 0.0)])
def test_channel_selection_matches_oracle(nsig, g2min):
    """The library's build-time selection keeps exactly the channels of the
    oracle's mask (the FP64 comparison is taken the same way on both sides),
    and the kept set has a valid layout."""
    import oracle
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    keep = oracle.select_channels(s, nsig, g2min)
    rp, partner, mode, chan = E.layout_host(s, energy_nsigma=nsig, g2_min=g2min)
    assert rp[-1] == 2 * keep.sum()
    kept = np.unique(chan)
    assert np.array_equal(kept, np.nonzero(keep)[0])
    assert np.all(np.bincount(chan, minlength=s.n_channels)[keep] == 2)
    _check_layout(oracle.subset(s, keep))


def test_selection_of_every_channel_and_option_errors():
    s = synth.two_state_system(dE=0.07, hw=0.03, g2=2e-3, sigma=0.008)
    rp, partner, *_ = E.layout_host(s, energy_nsigma=4.9)
    assert rp.tolist() == [0, 0, 0] and partner.size == 0
    rp, *_ = E.layout_host(s, energy_nsigma=5.1)
    assert rp.tolist() == [0, 1, 2]
    with pytest.raises(E.EphbteError, match="energy_nsigma"):
        E.layout_host(s, energy_nsigma=-1.0)
    with pytest.raises(E.EphbteError, match="g2_min"):
        E.layout_host(s, g2_min=float("nan"))
    lib = E.load_library()
    pr, keep = binding._problem(s, binding.F64, -1)
    o = binding.BuildOpts()
    o.reserved[1] = 1
    rp = np.zeros(3, np.int64)
    assert lib.ephbte_layout_host(ctypes.byref(pr), ctypes.byref(o), rp.ctypes.data, None, None,
                                  None) == binding.INVALID_ARGUMENT
    assert "reserved" in E.last_error()


def test_elastic_modes_option():
    """hw = 0 is accepted only for modes flagged elastic, which must be 0 at
    every q; the flagged channels are laid out like any other."""
    s = synth.defect_system(4, with_phonons=True)
    e = s.meta["elastic_mode"]
    with pytest.raises(E.EphbteError, match="below 1e-6"):
        E.layout_host(s)
    rp, partner, mode, chan = E.layout_host(s, elastic_modes=1 << e)
    assert rp[-1] == 2 * s.n_channels
    assert np.array_equal(np.sort(np.unique(chan)), np.arange(s.n_channels))
    with pytest.raises(E.EphbteError, match="n_modes"):
        E.layout_host(s, elastic_modes=1 << s.n_modes)
    hw = s.hw.copy()
    hw[3, e] = 1e-3
    s2 = _mutate_sys(s, hw=hw)
    with pytest.raises(E.EphbteError, match="elastic mode must be 0"):
        E.layout_host(s2, elastic_modes=1 << e)
    # a phonon mode flagged elastic has nonzero energies
    with pytest.raises(E.EphbteError, match="elastic mode must be 0"):
        E.layout_host(s, elastic_modes=(1 << e) | 1)


def _mutate_sys(s, **kw):
    import copy
    r = copy.copy(s)
    for k, v in kw.items():
        setattr(r, k, v)
    return r


def test_repeated_k_band_is_accepted():
    """Block-diagonal subsystems may hold the same (k, band); the layout is
    built (only the field term would be unavailable)."""
    s = synth.multiband_system()
    b = s.state_band.copy()
    same_k = np.nonzero(s.state_k == s.state_k[0])[0]
    assert same_k.size >= 2
    b[same_k[1]] = b[same_k[0]]
    rp, *_ = E.layout_host(_mutate_sys(s, state_band=b))
    assert rp[-1] == 2 * s.n_channels
    lib = E.load_library()
    r = np.zeros(3)
    assert lib.ephbte_set_field(None, r.ctypes.data) == binding.INVALID_ARGUMENT


def _bad(system, match):
    with pytest.raises(E.EphbteError, match=match) as ei:
        E.layout_host(system)
    return ei.value.status


def _mutate(**kw):
    s = synth.multiband_system()
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_validation_errors():
    base = synth.multiband_system()
    i, j = base.ch_i.copy(), base.ch_j.copy()
    j2 = j.copy()
    j2[3] = i[3]
    assert _bad(_mutate(ch_j=j2), "i == j") == binding.INVALID_ARGUMENT
    i2 = i.copy()
    i2[0] = base.n_states
    _bad(_mutate(ch_i=i2), "out of range")
    nu = base.ch_nu.copy()
    nu[1] = 7
    _bad(_mutate(ch_nu=nu), "mode index")
    g = base.g2.copy()
    g[2] = -1.0
    _bad(_mutate(g2=g), "finite and >= 0")
    g[2] = np.nan
    _bad(_mutate(g2=g), "finite and >= 0")
    _bad(_mutate(sigma=0.0), "sigma")
    _bad(_mutate(qgrid=(4, 3, 3)), "divide")
    # a pair from two different cosets of the q grid
    kc = synth.grid_coords(base.kgrid)[base.state_k]
    coset = synth.linear_index(kc % 2, (2, 2, 2))
    a = 0
    b = int(np.nonzero(coset != coset[0])[0][0])
    _bad(_mutate(ch_i=np.append(i, a).astype(np.int32), ch_j=np.append(j, b).astype(np.int32),
                 ch_nu=np.append(base.ch_nu, 1).astype(np.int8), g2=np.append(base.g2, 1e-3)),
         "q-grid vector")
    # acoustic mode at q = 0 (same k, different band)
    same_k = np.nonzero(base.state_k == base.state_k[0])[0]
    assert same_k.size >= 2
    _bad(_mutate(ch_i=np.append(i, same_k[0]).astype(np.int32),
                 ch_j=np.append(j, same_k[1]).astype(np.int32),
                 ch_nu=np.append(base.ch_nu, 0).astype(np.int8), g2=np.append(base.g2, 1e-3)),
         "below 1e-6")
    # duplicate channel, given in the other orientation
    _bad(_mutate(ch_i=np.append(i, j[5]).astype(np.int32), ch_j=np.append(j, i[5]).astype(np.int32),
                 ch_nu=np.append(base.ch_nu, base.ch_nu[5]).astype(np.int8),
                 g2=np.append(base.g2, 1e-3)), "duplicate")
    hw = base.hw.copy()
    hw[1, 2] *= 1.5
    _bad(_mutate(hw=hw), "even in q")
    sk = base.state_k.copy()
    sk[0] = 10 ** 6
    _bad(_mutate(state_k=sk), "state_k")


def test_bad_dtype_and_validation_precede_device_use():
    lib = E.load_library()
    s = synth.multiband_system()
    pr, keep = binding._problem(s, 3, 0)
    h = ctypes.c_void_p()
    assert lib.ephbte_build_channels(ctypes.byref(pr), None, ctypes.byref(h)) == binding.UNSUPPORTED_DTYPE
    g = s.g2.copy()
    g[0] = -1
    s.g2 = g
    pr, keep = binding._problem(s, binding.F64, 0)
    # invalid input is reported as such even on a machine without a GPU
    assert lib.ephbte_build_channels(ctypes.byref(pr), None, ctypes.byref(h)) == binding.INVALID_ARGUMENT
    assert h.value is None


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    s = synth.two_state_system()
    plan = binding.Plan.__new__(binding.Plan)
    plan.handle = None
    plan.n_states, plan.n_channels, plan.n_modes, plan.n_q = 2, 1, 1, 2
    plan.dtype, plan.device = binding.F64, 0
    with pytest.raises(TypeError, match="CUDA"):
        E.collision_integral(plan, torch.zeros(2, dtype=torch.float64),
                             torch.zeros(2, 1, dtype=torch.float64))
