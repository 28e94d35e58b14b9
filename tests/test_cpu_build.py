"""The library's kernels and host code built for the CPU (g++ with
AddressSanitizer and UndefinedBehaviorSanitizer, the HIP runtime replaced by
tests/cpu_build/hip/hip_runtime.h), run on small systems and compared with
the oracle.

This checks, without a GPU, that every index a kernel forms stays inside the
buffer it reads or writes (each device buffer is a separate host allocation,
dynamic LDS is poisoned beyond the launch's size), that the host code
launches what the kernels assume, and that the arithmetic is the oracle's.
It covers the entry points' B = 1 forms (single-copy and per-row), the
batched forms (B >= 8, with the DPP and shuffle exchanges emulated lane by
lane), channel selection at build, elastic mechanisms, per-vector phonon
baths, an uneven group of systems, new |g|^2 loaded into a plan, the
autotuner and its cache, RK4 eager and replayed from a captured graph, the RK4 adjoint, the
transport iteration, the phonon-side rate, the field term of Eq. 1 and the
coupled electron-phonon step.  Fresh device memory and LDS can be filled with
random bytes and workgroups run in any order, so that a result depending on
unwritten memory or on scheduling shows up here.

The CPU build is a separate executable made here for tests only; the package
never loads it, and the GPU tests run the HIP library itself.
"""
import hashlib
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2511_03683_amd", "csrc")
SHIM = os.path.join(HERE, "cpu_build")
SOURCES = ("api.hip", "kernels.hpp", "layout.hpp", "layout.cpp")
TOL64, TOL32 = 1e-10, 1e-5
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _digest():
    h = hashlib.sha256()
    for p in [os.path.join(CSRC, s) for s in SOURCES] + [
            os.path.join(ROOT, "include", "ephbte.h"),
            os.path.join(SHIM, "hip", "hip_runtime.h"), os.path.join(SHIM, "driver.cpp")]:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


@pytest.fixture(scope="module")
def driver():
    """Compile the CPU build once per source state (about a minute)."""
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ is not available")
    root = os.path.join(SHIM, "_build")
    digest = _digest()
    bdir = os.path.join(root, digest)
    exe = os.path.join(bdir, "driver")
    if os.path.exists(exe):
        return exe
    if os.path.isdir(root):   # builds of earlier source states
        for old in os.listdir(root):
            if old != digest:
                shutil.rmtree(os.path.join(root, old), ignore_errors=True)
    src = os.path.join(bdir, "src")
    os.makedirs(src, exist_ok=True)
    for s in SOURCES:
        with open(os.path.join(CSRC, s)) as fh:
            text = fh.read()
        # dynamic LDS comes from the stand-in's buffer
        text = text.replace("extern __shared__ __align__(16) unsigned char smem[];",
                            "unsigned char *smem = emu::dyn_smem();")
        with open(os.path.join(src, s), "w") as fh:
            fh.write(text)
    cmd = [cxx, "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", SHIM, "-I", src, "-I", os.path.join(ROOT, "include"),
           "-o", exe + ".tmp", os.path.join(SHIM, "driver.cpp"), os.path.join(src, "layout.cpp"),
           "-lpthread"]
    subprocess.run(cmd, check=True, timeout=900)
    os.replace(exe + ".tmp", exe)
    return exe


def _write(folder, s, dtype="f64", **kw):
    arrs = dict(state_k=np.asarray(s.state_k, np.int32), state_band=np.asarray(s.state_band, np.int8),
                eps=np.asarray(s.eps, np.float64), hw=np.asarray(s.hw, np.float64),
                ci=np.asarray(s.ch_i, np.int32), cj=np.asarray(s.ch_j, np.int32),
                cn=np.asarray(s.ch_nu, np.int8), g2=np.asarray(s.g2, np.float64))
    meta = dict(S=s.n_states, nm=s.n_modes, nch=s.n_channels, kgrid=list(s.kgrid),
                qgrid=list(s.qgrid), sigma=s.sigma, nq=s.n_q_norm, dtype=1 if dtype == "f32" else 2)
    for k, v in kw.items():
        if isinstance(v, np.ndarray):
            arrs[k] = np.ascontiguousarray(v, np.float64)
        else:
            meta[k] = v
    for k, v in arrs.items():
        v.tofile(os.path.join(folder, k + ".bin"))
    with open(os.path.join(folder, "meta.txt"), "w") as fh:
        for k, v in meta.items():
            vals = v if isinstance(v, (list, tuple)) else [v]
            fh.write(k + " " + " ".join(repr(float(x)) for x in vals) + "\n")


def _run(driver, folder, mode, order=None, fill=None):
    env = dict(ENV)
    if order is not None:
        env["CPU_BUILD_ORDER"] = order
    if fill is not None:
        env["CPU_BUILD_FILL"] = fill
    r = subprocess.run([driver, mode, str(folder)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, f"{mode}: exit {r.returncode}\n{r.stdout}\n{r.stderr[-4000:]}"
    return r


def _out(folder, name, shape=None):
    a = np.fromfile(os.path.join(folder, "out_" + name + ".bin"))
    return a.reshape(shape) if shape is not None else a


def nerr(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / max(np.abs(ref).max(), 1e-300))


def _round32(s):
    import copy
    r = copy.copy(s)
    r.eps = s.eps.astype(np.float32).astype(np.float64)
    r.hw = s.hw.astype(np.float32).astype(np.float64)
    r.g2 = s.g2.astype(np.float32).astype(np.float64)
    return r


@pytest.mark.parametrize("layout,dtype,fexp,order", [(2, "f64", 0, 1), (1, "f64", 0, 1), (2, "f32", 0, 1),
                                                     (3, "f64", 1, 1), (3, "f64", 2, 1), (3, "f32", 0, 1),
                                                     (3, "f64", 1, 2), (2, "f64", 0, 2), (1, "f32", 0, 2)])
def test_forward_single_vector(driver, tmp_path, layout, dtype, fexp, order):
    """Single-copy (layout 2: one entry per channel; layout 3: pair records,
    FP64 Gaussians from the table or the polynomial exponential) and per-row
    (layout 1) forward passes, B = 1, with the {hw, N} table in either order."""
    s = synth.multiband_system()
    f = synth.random_occupations(s, 3)
    nph = s.nph(300.0)
    _write(tmp_path, s, dtype, f=f, nph=nph, B=1, layout=layout, fp64_exp=fexp, table_order=order)
    _run(driver, tmp_path, "forward")
    # one launch of the forward kernel, bracketed by the timing events
    assert _out(tmp_path, "timing")[1] == 1
    if dtype == "f64":
        assert nerr(_out(tmp_path, "I"), oracle.collision(s, f, nph)) <= TOL64
    else:
        r = _round32(s)
        f32, n32 = f.astype(np.float32).astype(np.float64), nph.astype(np.float32).astype(np.float64)
        assert nerr(_out(tmp_path, "I"), oracle.collision(r, f32, n32)) <= TOL32


@pytest.mark.parametrize("B,order", [(3, 1), (9, 1), (3, 2), (9, 2)])
def test_forward_batched(driver, tmp_path, B, order):
    """Per-row pass for B < 8 and the batched pass (LDS tiles, run merge over
    lanes) for B >= 8, every column against the oracle, with the {hw, N}
    table in either order."""
    s = synth.multiband_system()
    F = np.stack([synth.random_occupations(s, 10 + b) for b in range(B)])
    nph = s.nph(300.0)
    _write(tmp_path, s, f=F, nph=nph, B=B, table_order=order)
    _run(driver, tmp_path, "forward")
    got = _out(tmp_path, "I", (B, s.n_states))
    for b in range(B):
        assert nerr(got[b], oracle.collision(s, F[b], nph)) <= TOL64, b


@pytest.mark.parametrize("B,order", [(1, 1), (9, 1), (1, 2), (9, 2)])
def test_vjp(driver, tmp_path, B, order):
    """Reverse pass, B = 1 (per-row kernel) and batched (DPP sums over the
    vectors): dL/df per vector and dL/d|g|^2 summed over the vectors, with
    the {hw, N} table in either order."""
    s = synth.multiband_system()
    F = np.stack([synth.random_occupations(s, 20 + b) for b in range(B)])
    lam = np.random.default_rng(4).normal(size=(B, s.n_states))
    nph = s.nph(300.0)
    _write(tmp_path, s, f=F, lam=lam, nph=nph, B=B, table_order=order)
    _run(driver, tmp_path, "vjp")
    gf = _out(tmp_path, "gf", (B, s.n_states))
    gg = _out(tmp_path, "gg2")
    rg = np.zeros(s.n_channels)
    for b in range(B):
        rf_b, rg_b = oracle.collision_vjp(s, F[b], nph, lam[b])
        assert nerr(gf[b], rf_b) <= TOL64, b
        rg += rg_b
    assert nerr(gg, rg) <= TOL64


def test_rt_step_and_graph(driver, tmp_path):
    """RK4 steps through the single-copy pass, eager and replayed from a
    captured graph (bitwise equal)."""
    s = synth.multiband_system()
    f0 = synth.random_occupations(s, 7)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f0, nph=nph, B=1, dt=0.5, steps=3)
    _run(driver, tmp_path, "rt")
    ref = f0.copy()
    for _ in range(3):
        ref = oracle.rk4_step(s, ref, nph, 0.5)
    got = _out(tmp_path, "f")
    assert nerr(got - f0, ref - f0) <= TOL64
    assert np.array_equal(_out(tmp_path, "f_graph"), got)


def test_rt_adjoint(driver, tmp_path):
    s = synth.multiband_system(n_k=10, seed=23)
    f0 = synth.random_occupations(s, 9) * 0.8 + 0.1
    nph = s.nph(300.0)
    gT = np.random.default_rng(5).normal(size=s.n_states)
    _write(tmp_path, s, f=f0, gT=gT, nph=nph, dt=0.5, steps=4, ce=2)
    _run(driver, tmp_path, "adjoint")
    _, rf, rg = oracle.rk4_trajectory_grad(s, f0, nph, 0.5, 4, gT)
    assert nerr(_out(tmp_path, "gf"), rf) <= 1e-9
    assert nerr(_out(tmp_path, "gg2"), rg) <= 1e-9


def test_transport(driver, tmp_path):
    s = synth.tb_system(kn=12, qn=6, target_states=120, sigma=0.05)
    T = 300.0
    f0 = synth.fermi_dirac(s.eps, -0.1, T)
    nph = s.nph(T)
    _write(tmp_path, s, f=f0, vel=np.asarray(s.vel), nph=nph, T=T, tol=0.0, max_iter=5)
    _run(driver, tmp_path, "transport")
    ref = oracle.transport_solve(s, f0, s.vel, T, nph, max_iter=5, stop_on_tol=False)
    assert nerr(_out(tmp_path, "mob", (3, 3)), ref["mu"]) <= TOL64
    assert nerr(_out(tmp_path, "x", (s.n_states, 3)), ref["x"]) <= TOL64


@pytest.mark.parametrize("name", ["multiband", "random", "tb", "defect"])
def test_phonon_rate(driver, tmp_path, name):
    """dN/dt over the pair records bucketed by {q, -q} against the oracle's
    channel loop; the defect system's elastic mechanism exchanges no phonon,
    so its channels are left out (its bins are zero)."""
    s = {"multiband": synth.multiband_system, "random": synth.random_channel_system,
         "tb": lambda: synth.tb_system(kn=24, qn=12, target_states=400),
         "defect": lambda: synth.defect_system(5)}[name]()
    f = synth.random_occupations(s, 50)
    nph = s.nph(300.0)
    kw, keep = {}, np.ones(s.n_channels, bool)
    if name == "defect":
        e = s.meta["elastic_mode"]
        kw["elastic_modes"] = 1 << e
        keep = np.asarray(s.ch_nu) != e
    _write(tmp_path, s, f=f, nph=nph, **kw)
    _run(driver, tmp_path, "phonon")
    ref = oracle.phonon_rate(oracle.subset(s, keep), f, nph)
    got = _out(tmp_path, "rate", ref.shape)
    if name == "defect":
        assert np.all(got[:, s.meta["elastic_mode"]] == 0.0)
    assert nerr(got, ref) <= TOL64


@pytest.mark.parametrize("B", [1, 3, 9])
def test_field_term(driver, tmp_path, B):
    """The field term of Eq. 1 in the RK4 stage epilogues (single-copy,
    per-row and batched forward passes), eager and graph."""
    s = synth.multiband_system()
    rates = [0.06, -0.035, 0.02]
    F = np.stack([synth.random_occupations(s, 30 + b) for b in range(B)])
    nph = s.nph(300.0)
    _write(tmp_path, s, f=F, nph=nph, B=B, dt=1.0, steps=4, rates=rates)
    _run(driver, tmp_path, "field")
    got = _out(tmp_path, "f", (B, s.n_states))
    for b in range(B):
        ref = F[b].copy()
        for _ in range(4):
            ref = oracle.rk4_step(s, ref, nph, 1.0, rates=np.array(rates))
        assert nerr(got[b] - F[b], ref - F[b]) <= 1e-9, b
    assert np.array_equal(_out(tmp_path, "f_graph", (B, s.n_states)), got)


@pytest.mark.parametrize("name", ["multiband", "tb24"])
def test_coupled_step(driver, tmp_path, name):
    """The coupled electron-phonon RK4 step."""
    s = synth.multiband_system() if name == "multiband" else \
        synth.tb_system(kn=24, qn=12, target_states=400)
    f0 = 0.1 + 0.8 * synth.random_occupations(s, 52)
    N0 = s.nph(300.0) * 1.5
    _write(tmp_path, s, f=f0, nph=N0, dt=1.0, steps=3)
    _run(driver, tmp_path, "coupled")
    rf, rN = f0, N0
    for _ in range(3):
        rf, rN = oracle.rk4_coupled_step(s, rf, rN, 1.0)
    assert nerr(_out(tmp_path, "f") - f0, rf - f0) <= 1e-9
    assert nerr(_out(tmp_path, "N", rN.shape) - N0, rN - N0) <= 1e-9


def test_channel_selection(driver, tmp_path):
    """A plan built with the energy window and |g|^2 floor computes Eq. 2
    over the oracle's kept channels; removed channels get zero gradients."""
    s = synth.tb_system(kn=12, qn=6, target_states=120, sigma=0.05)
    nsig, g2min = 2.5, 5e-4
    keep = oracle.select_channels(s, nsig, g2min)
    assert 0 < keep.sum() < s.n_channels
    sub = oracle.subset(s, keep)
    f = synth.random_occupations(s, 31)
    lam = np.random.default_rng(8).normal(size=s.n_states)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f, lam=lam, nph=nph, energy_nsigma=nsig, g2_min=g2min, gg2_fill=7.0)
    _run(driver, tmp_path, "forward")
    assert nerr(_out(tmp_path, "I"), oracle.collision(sub, f, nph)) <= TOL64
    _run(driver, tmp_path, "vjp")
    rf, rg = oracle.collision_vjp(sub, f, nph, lam)
    gg = _out(tmp_path, "gg2")
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64
    assert np.all(gg[~keep] == 0.0)
    assert nerr(gg[keep], rg) <= TOL64


def test_elastic_mechanism(driver, tmp_path):
    """A defect mechanism flagged elastic beside phonon modes."""
    s = synth.defect_system(6, with_phonons=True)
    e = s.meta["elastic_mode"]
    f = synth.random_occupations(s, 14)
    lam = np.random.default_rng(9).normal(size=s.n_states)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f, lam=lam, nph=nph, elastic_modes=1 << e)
    _run(driver, tmp_path, "forward")
    assert nerr(_out(tmp_path, "I"), oracle.collision(s, f, nph)) <= TOL64
    _run(driver, tmp_path, "vjp")
    rf, rg = oracle.collision_vjp(s, f, nph, lam)
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64
    assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64


@pytest.mark.parametrize("B,dtype", [(3, "f64"), (9, "f64"), (70, "f64"), (9, "f32")])
def test_bath_per_vector(driver, tmp_path, B, dtype):
    """nph [B, Nq, n_modes]: each vector against the oracle with its own bath,
    forward and reverse; B >= 8 runs the batched passes with the baths in
    groups of 64 vectors (70: two groups), under random fills of fresh
    memory."""
    s = synth.multiband_system()
    temps = [150.0 + 37.0 * b for b in range(B)]
    F = np.stack([synth.random_occupations(s, 40 + b) for b in range(B)])
    NPH = np.stack([s.nph(T) for T in temps])
    L = np.random.default_rng(5).normal(size=(B, s.n_states))
    _write(tmp_path, s, dtype, f=F, lam=L, nph=NPH, B=B, nph_per_batch=1)
    _run(driver, tmp_path, "forward", fill="random:%d" % B)
    got = _out(tmp_path, "I", (B, s.n_states))
    if dtype == "f32":
        r = _round32(s)
        for b in range(B):
            fb, nb = F[b].astype(np.float32).astype(np.float64), NPH[b].astype(np.float32).astype(np.float64)
            ref = oracle.collision(r, fb, nb)
            rin, rout = oracle.collision_inout(r, fb, nb)
            scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
            assert np.abs(got[b] - ref).max() / scale <= TOL32, b
        return
    for b in range(B):
        assert nerr(got[b], oracle.collision(s, F[b], NPH[b])) <= TOL64, b
    _run(driver, tmp_path, "vjp", fill="random:%d" % (B + 1))
    gf = _out(tmp_path, "gf", (B, s.n_states))
    rg = 0
    for b in range(B):
        rf_b, rg_b = oracle.collision_vjp(s, F[b], NPH[b], L[b])
        assert nerr(gf[b], rf_b) <= TOL64, b
        rg = rg + rg_b
    assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64


@pytest.mark.parametrize("mode,B,dtype", [("forward", 1, "f64"), ("forward", 1, "f32"),
                                          ("forward", 9, "f64"), ("vjp", 1, "f64"),
                                          ("vjp", 9, "f64"), ("phonon", 1, "f64")])
def test_results_do_not_depend_on_scheduling(driver, tmp_path, mode, B, dtype):
    """Bitwise the same outputs when workgroups, and the work-items inside each,
    run in forward, reverse or shuffled order: the partner-side and phonon-bin
    sums are integer atomics and every floating-point sum has a fixed order."""
    s = synth.multiband_system()
    F = np.stack([synth.random_occupations(s, 60 + b) for b in range(B)])
    lam = np.random.default_rng(12).normal(size=(B, s.n_states))
    _write(tmp_path, s, dtype, f=F, lam=lam, nph=s.nph(300.0), B=B)
    names = {"forward": ["I"], "vjp": ["gf", "gg2"], "phonon": ["rate"]}[mode]
    outs = []
    for order in ("forward", "reverse", "shuffle:1", "shuffle:2"):
        _run(driver, tmp_path, mode, order)
        outs.append([_out(tmp_path, n) for n in names])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


TUNINGS = [dict(chunk_entries=37, block_threads=64),
           dict(chunk_entries=256, block_threads=128, xcd_map=2, layout=1),
           dict(block_threads=512, tile_entries=500, xcd_map=1),
           dict(chunk_entries=37, layout=1, tile_entries=100)]


@pytest.mark.parametrize("k", range(len(TUNINGS)))
def test_tuning_variants(driver, tmp_path, k):
    """Chunk sizes that split destinations (chunk partials summed in order),
    block sizes, tile targets and XCD maps: the forward pass (B = 1 and the
    batched pass with 16-partner sub-tiles) and the reverse pass against the
    oracle."""
    tune = TUNINGS[k]
    s = synth.random_channel_system(n_states=60, n_channels=900, seed=3)
    F = np.stack([synth.random_occupations(s, 70 + b) for b in range(9)])
    lam = np.random.default_rng(13).normal(size=(9, s.n_states))
    nph = s.nph(300.0)
    _write(tmp_path, s, f=F[:1], lam=lam[:1], nph=nph, B=1, **tune)
    _run(driver, tmp_path, "forward")
    assert nerr(_out(tmp_path, "I"), oracle.collision(s, F[0], nph)) <= TOL64
    _run(driver, tmp_path, "vjp")
    rf, rg = oracle.collision_vjp(s, F[0], nph, lam[0])
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64 and nerr(_out(tmp_path, "gg2"), rg) <= TOL64
    _write(tmp_path, s, f=F, nph=nph, B=9, batch_partners=16, **tune)
    _run(driver, tmp_path, "forward")
    got = _out(tmp_path, "I", (9, s.n_states))
    for b in range(9):
        assert nerr(got[b], oracle.collision(s, F[b], nph)) <= TOL64, b


def test_field_term_in_the_adjoint(driver, tmp_path):
    """The discrete RK4 adjoint with the field term (its transpose in the
    adjoint stage epilogues), against the oracle's adjoint with drift."""
    s = synth.multiband_system(n_k=10, seed=23)
    f0 = synth.random_occupations(s, 9) * 0.8 + 0.1
    nph = s.nph(300.0)
    rates = [0.06, -0.035, 0.02]
    gT = np.random.default_rng(6).normal(size=s.n_states)
    _write(tmp_path, s, f=f0, gT=gT, nph=nph, dt=1.0, steps=4, ce=2, rates=rates)
    _run(driver, tmp_path, "adjoint")
    _, rf, rg = oracle.rk4_trajectory_grad(s, f0, nph, 1.0, 4, gT, rates=np.array(rates))
    assert nerr(_out(tmp_path, "gf"), rf) <= 1e-9
    assert nerr(_out(tmp_path, "gg2"), rg) <= 1e-9


@pytest.mark.parametrize("mode,B", [("forward", 9), ("vjp", 1), ("vjp", 9)])
def test_fp32_passes(driver, tmp_path, mode, B):
    """FP32 batched forward and reverse passes against the FP64 oracle on the
    FP32-rounded inputs."""
    s = synth.multiband_system()
    r = _round32(s)
    F = np.stack([synth.random_occupations(s, 80 + b) for b in range(B)]).astype(np.float32).astype(np.float64)
    lam = np.random.default_rng(14).normal(size=(B, s.n_states)).astype(np.float32).astype(np.float64)
    nph = s.nph(300.0).astype(np.float32).astype(np.float64)
    _write(tmp_path, s, "f32", f=F, lam=lam, nph=nph, B=B)
    _run(driver, tmp_path, mode)
    if mode == "forward":
        got = _out(tmp_path, "I", (B, s.n_states))
        for b in range(B):
            ref = oracle.collision(r, F[b], nph)
            rin, rout = oracle.collision_inout(r, F[b], nph)
            scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
            assert np.abs(got[b] - ref).max() / scale <= TOL32, b
    else:
        gf = _out(tmp_path, "gf", (B, s.n_states))
        rg = 0
        for b in range(B):
            rf_b, rg_b = oracle.collision_vjp(r, F[b], nph, lam[b])
            assert nerr(gf[b], rf_b) <= TOL32, b
            rg = rg + rg_b
        assert nerr(_out(tmp_path, "gg2"), rg) <= TOL32


UNWRITTEN_CASES = [("forward", dict(B=1)), ("forward", dict(B=1, layout=1)), ("forward", dict(B=9)),
                   ("forward", dict(B=1, table_order=2)), ("vjp", dict(B=1, table_order=2)),
                   ("vjp", dict(B=1)), ("vjp", dict(B=9)), ("phonon", dict()),
                   ("rt", dict(B=1, dt=0.5, steps=2)),
                   ("field", dict(B=1, dt=1.0, steps=2, rates=[0.06, -0.035, 0.02])),
                   ("coupled", dict(dt=1.0, steps=2))]


@pytest.mark.parametrize("k", range(len(UNWRITTEN_CASES)))
def test_results_do_not_read_unwritten_memory(driver, tmp_path, k):
    """Fresh device memory and each workgroup's LDS filled with random bytes
    (two seeds) instead of fixed patterns: the outputs are bitwise the same,
    so no result depends on memory that nothing wrote (on the GPU, LDS holds
    whatever the previous workgroup left)."""
    mode, kw = UNWRITTEN_CASES[k]
    s = synth.multiband_system()
    B = kw.get("B", 1)
    F = np.stack([0.1 + 0.8 * synth.random_occupations(s, 90 + b) for b in range(B)])
    lam = np.random.default_rng(15).normal(size=(B, s.n_states))
    _write(tmp_path, s, f=F, lam=lam, nph=s.nph(300.0), **kw)
    names = {"forward": ["I"], "vjp": ["gf", "gg2"], "phonon": ["rate"], "rt": ["f", "f_graph"],
             "field": ["f", "f_graph"], "coupled": ["f", "N"]}[mode]
    outs = []
    for fill in (None, "random:1", "random:2"):
        _run(driver, tmp_path, mode, fill=fill)
        outs.append([_out(tmp_path, n) for n in names])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


EMPTY_WINDOW_CASES = [("forward", dict(B=1)), ("forward", dict(B=1, layout=1)), ("vjp", dict(B=1)),
                      ("rt", dict(B=1, dt=0.5, steps=2)), ("transport", dict())]


@pytest.mark.parametrize("k", range(len(EMPTY_WINDOW_CASES)))
def test_masked_lanes_ignore_empty_windows(driver, tmp_path, k):
    """Tiles whose chunks hold no entries are given an empty partner window
    (nothing staged in LDS) and LDS is filled with random bytes: the masked
    lanes of those chunks must form their table index and operands without
    the window, so the outputs are bitwise those of the plain run."""
    mode, kw = EMPTY_WINDOW_CASES[k]
    s = synth.multiband_system()
    B = kw.get("B", 1)
    F = np.stack([0.1 + 0.8 * synth.random_occupations(s, 120 + b) for b in range(B)])
    lam = np.random.default_rng(19).normal(size=(B, s.n_states))
    if mode == "transport":
        f0 = synth.fermi_dirac(s.eps, float(np.min(s.eps)) - 0.05, 300.0)
        vel = np.random.default_rng(20).normal(size=(s.n_states, 3)) * 1e5
        _write(tmp_path, s, f=f0, vel=vel, nph=s.nph(300.0), T=300.0, tol=0.0, max_iter=4)
        names = ["x", "mob"]
    else:
        _write(tmp_path, s, f=F, lam=lam, nph=s.nph(300.0), **kw)
        names = {"forward": ["I"], "vjp": ["gf", "gg2"], "rt": ["f", "f_graph"]}[mode]
    _run(driver, tmp_path, mode)
    ref = [_out(tmp_path, n) for n in names]
    with open(os.path.join(tmp_path, "meta.txt"), "a") as fh:
        fh.write("empty_windows 1.0\n")
    for fill in ("random:21", "random:22"):
        _run(driver, tmp_path, mode, fill=fill)
        assert _out(tmp_path, "emptied")[0] > 0, "the system has tiles without entries"
        for n, a in zip(names, ref):
            assert np.array_equal(_out(tmp_path, n), a), (mode, n, fill)


SWEEP_SYSTEMS = {
    "parabolic4": lambda: synth.parabolic_system(4),
    "random_order": lambda: synth.random_channel_system(n_states=60, n_channels=900, seed=3),
    "tb12": lambda: synth.tb_system(kn=12, qn=6, target_states=120, sigma=0.05),
    "defect": lambda: synth.defect_system(6, with_phonons=True),
}


@pytest.mark.parametrize("name", sorted(SWEEP_SYSTEMS))
def test_other_systems_do_not_read_unwritten_memory(driver, tmp_path, name):
    """The random-fill check on four more systems (dense, unstructured,
    multi-band tight-binding, one elastic mechanism): forward at B = 1 and 9,
    reverse at B = 1, bitwise the same under two random fills."""
    s = SWEEP_SYSTEMS[name]()
    extra = dict(elastic_modes=1 << s.meta["elastic_mode"]) if name == "defect" else {}
    for mode, B in (("forward", 1), ("forward", 9), ("vjp", 1)):
        F = np.stack([0.05 + 0.9 * synth.random_occupations(s, 100 + b) for b in range(B)])
        lam = np.random.default_rng(16).normal(size=(B, s.n_states))
        _write(tmp_path, s, f=F, lam=lam, nph=s.nph(300.0), B=B, **extra)
        names = ["I"] if mode == "forward" else ["gf", "gg2"]
        outs = []
        for fill in (None, "random:11", "random:12"):
            _run(driver, tmp_path, mode, fill=fill)
            outs.append([_out(tmp_path, n) for n in names])
        for o in outs[1:]:
            for a, b in zip(outs[0], o):
                assert np.array_equal(a, b), (name, mode, B)


def test_update_g2(driver, tmp_path):
    """New |g|^2 loaded into a built plan (caller order): the forward pass
    follows them."""
    s = synth.multiband_system()
    f = synth.random_occupations(s, 17)
    nph = s.nph(300.0)
    g2n = s.g2 * np.random.default_rng(18).uniform(0.5, 2.0, size=s.n_channels)
    _write(tmp_path, s, f=f, nph=nph, g2_new=g2n)
    _run(driver, tmp_path, "update_g2")
    assert nerr(_out(tmp_path, "I"), oracle.collision(s, f, nph, g2=g2n)) <= TOL64
    ref = oracle.phonon_rate(s, f, nph, g2=g2n)
    assert nerr(_out(tmp_path, "rate", ref.shape), ref) <= TOL64


@pytest.mark.parametrize("B", [1, 9])
def test_autotune_with_cache(driver, tmp_path, B):
    """The autotuner times its candidates, writes the choice to the cache file,
    and the second call reads the same choice back; the tuned plan still
    matches the oracle."""
    import json
    s = synth.multiband_system()
    F = np.stack([synth.random_occupations(s, 110 + b) for b in range(B)])
    nph = s.nph(300.0)
    _write(tmp_path, s, f=F, nph=nph, B=B)
    _run(driver, tmp_path, "autotune")
    t = _out(tmp_path, "tune")
    assert np.array_equal(t[:3], t[3:])
    with open(tmp_path / "tune.json") as fh:
        cache = json.load(fh)
    assert len(cache) == 1
    got = _out(tmp_path, "I", (B, s.n_states))
    for b in range(B):
        assert nerr(got[b], oracle.collision(s, F[b], nph)) <= TOL64, b


def test_grouped_uneven_systems(driver, tmp_path):
    """Four systems of 100 .. 3000 channels concatenated into one problem and
    evaluated by one forward pass, every state against the oracle."""
    base = synth.tb_system(kn=12, qn=6, target_states=120, sigma=0.05, with_channels=False)
    s = synth.grouped_system(n_systems=4, ch_min=100, ch_max=3000, base=base)
    f = synth.random_occupations(s, 19)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f, nph=nph)
    _run(driver, tmp_path, "forward")
    assert nerr(_out(tmp_path, "I"), oracle.collision(s, f, nph)) <= TOL64


@pytest.mark.parametrize("name,tune", [("multiband", {}), ("multiband", dict(chunk_entries=5)),
                                       ("multiband", dict(pair_order=2)), ("tb12", dict(pair_window=64)),
                                       ("tb12", dict(pair_rows=16)),
                                       ("parabolic4", {}), ("random_order", dict(chunk_entries=37)),
                                       ("tb12", {}), ("defect", {}), ("grouped", {})])
def test_tile_tables(driver, tmp_path, name, tune):
    """Every LDS tile of the four tile tables (forward, reverse/transport,
    single copy, pair records) stages 1 .. cap states, its window holds every
    partner of its chunks, and the tiles cover the chunks in order; the
    q-ordered pair tiles hold every record once, in the order of their q."""
    if name == "multiband":
        s = synth.multiband_system()
    elif name == "grouped":
        base = synth.tb_system(kn=12, qn=6, target_states=120, sigma=0.05, with_channels=False)
        s = synth.grouped_system(n_systems=4, ch_min=100, ch_max=3000, base=base)
    else:
        s = SWEEP_SYSTEMS[name]()
    if name == "defect":
        tune = dict(tune, elastic_modes=1 << s.meta["elastic_mode"])
    _write(tmp_path, s, f=synth.random_occupations(s, 1), nph=s.nph(300.0), **tune)
    _run(driver, tmp_path, "tiles")
    out = _out(tmp_path, "tiles")
    assert np.all(out[:4] == 0), out
    # q-ordered pair tiles, unless destination order was asked for
    n_q = -out[4]
    if tune.get("pair_order") == 2:
        assert n_q == 0, out
    elif name in ("multiband", "tb12", "parabolic4"):
        assert n_q > 0, out
        if not tune:   # every pair tile q-ordered: the phonon side's dL/df runs over them
            assert out[5] == 1, out


@pytest.mark.parametrize("name,layout,dtype", [("multiband", 2, "f64"), ("multiband", 1, "f64"),
                                               ("multiband", 2, "f32"), ("parabolic", 2, "f64"),
                                               ("random", 2, "f64")])
def test_allocation_free_pass(driver, tmp_path, name, layout, dtype):
    """The allocation-free forward pass (its table and partials in the
    library's static scratch, which holds random bytes here) gives bitwise
    the result of the plain pass and calls hipMalloc zero times."""
    s = {"multiband": synth.multiband_system, "parabolic": lambda: synth.parabolic_system(4),
         "random": synth.random_channel_system}[name]()
    f = 0.05 + 0.9 * synth.random_occupations(s, 11)
    nph = s.nph(300.0)
    _write(tmp_path, s, dtype, f=f, nph=nph, layout=layout)
    _run(driver, tmp_path, "noalloc", fill="random:5")
    I, J = _out(tmp_path, "I"), _out(tmp_path, "J")
    assert _out(tmp_path, "mallocs")[0] == 0
    assert np.array_equal(I, J)
    if dtype == "f64":
        assert nerr(J, oracle.collision(s, f, nph)) <= TOL64


def test_allocation_free_pass_rejects_large_tables(driver, tmp_path):
    """A phonon table larger than the static scratch (1024 x 1024 x 3 q
    points: 50 MB of {hw, N} in FP64) is refused before any work."""
    import dataclasses
    s = synth.two_state_system()
    q = (1024, 1024, 3)
    s = dataclasses.replace(s, kgrid=q, qgrid=q, hw=np.full((int(np.prod(q)), 1), 0.05),
                            n_q_norm=float(np.prod(q)))
    _write(tmp_path, s, f=np.array([0.3, 0.6]), nph=s.nph(300.0))
    r = subprocess.run([driver, "noalloc", str(tmp_path)], env=ENV, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 3
    assert "collision_integral_noalloc: status 1" in r.stderr and "bytes of scratch" in r.stderr


def _uneven_bath(s, seed):
    rng = np.random.default_rng(seed)
    return s.nph(300.0) * rng.uniform(0.5, 1.5, size=s.hw.shape)


@pytest.mark.parametrize("name,layout", [("multiband", 0), ("tb", 0), ("defect", 0), ("multiband", 1)])
def test_collision_vjp_nph(driver, tmp_path, name, layout):
    """dL/dN of L = lam . I over the records grouped by {q, -q}, against the
    oracle, on a bath that is not even in q (so that q and -q cannot be
    confused); the defect system's elastic channels count too."""
    s = {"multiband": synth.multiband_system, "tb": lambda: synth.tb_system(kn=24, qn=12, target_states=400),
         "defect": lambda: synth.defect_system(5)}[name]()
    f = synth.random_occupations(s, 61)
    N = _uneven_bath(s, 62)
    kw = {}
    if name == "defect":
        N[:, s.meta["elastic_mode"]] = 0.0
        kw["elastic_modes"] = 1 << s.meta["elastic_mode"]
    lam = np.random.default_rng(63).normal(size=s.n_states)
    _write(tmp_path, s, f=f, lam=lam, nph=N, layout=layout, **kw)
    _run(driver, tmp_path, "vjp_nph", fill="random:3")
    ref = oracle.collision_vjp_nph(s, f, N, lam)
    assert nerr(_out(tmp_path, "gN", ref.shape), ref) <= TOL64


@pytest.mark.parametrize("name,chunk", [("multiband", 0), ("tb", 0), ("defect", 0), ("tb", 50)])
def test_phonon_rate_vjp(driver, tmp_path, name, chunk):
    """Reverse of the phonon-side rate (dL/df over the destination layout,
    dL/dN and dL/d|g|^2 over the {q, -q} records) against the oracle, on a
    bath not even in q and a random bin adjoint; elastic channels get no
    |g|^2 gradient from it.  chunk splits destinations over several chunks."""
    s = {"multiband": synth.multiband_system, "tb": lambda: synth.tb_system(kn=24, qn=12, target_states=400),
         "defect": lambda: synth.defect_system(5)}[name]()
    f = synth.random_occupations(s, 71)
    N = _uneven_bath(s, 72)
    kw = {}
    keep = np.ones(s.n_channels, bool)
    if name == "defect":
        e = s.meta["elastic_mode"]
        N[:, e] = 0.0
        kw["elastic_modes"] = 1 << e
        keep = np.asarray(s.ch_nu) != e
    if chunk:
        kw["chunk_entries"] = chunk
    mu = np.random.default_rng(73).normal(size=N.shape)
    _write(tmp_path, s, f=f, mu=mu, nph=N, **kw)
    _run(driver, tmp_path, "phonon_vjp", fill="random:4")
    rf, rN, rg = oracle.phonon_rate_vjp(oracle.subset(s, keep), f, N, mu)
    gg = np.zeros(s.n_channels)
    gg[keep] = rg
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64
    assert nerr(_out(tmp_path, "gN", rN.shape), rN) <= TOL64
    assert nerr(_out(tmp_path, "gg2") - 0.25, gg) <= TOL64


@pytest.mark.parametrize("name,ce", [("multiband", 1), ("multiband", 2), ("tb", 3)])
def test_coupled_adjoint(driver, tmp_path, name, ce):
    """Gradients through three coupled RK4 steps against the oracle's discrete
    adjoint with every stage stored; checkpoints every ce steps."""
    s = {"multiband": synth.multiband_system, "tb": lambda: synth.tb_system(kn=24, qn=12, target_states=400)}[name]()
    f0 = 0.1 + 0.8 * synth.random_occupations(s, 81)
    N0 = s.nph(300.0) * 1.5
    rng = np.random.default_rng(82)
    a = rng.normal(size=s.n_states)
    b = oracle.even_in_q(s, rng.normal(size=N0.shape))
    dt, n = 1.0, 3
    _, _, rf, rN, rg = oracle.rk4_coupled_trajectory_grad(s, f0, N0, dt, n, a, b)
    _write(tmp_path, s, f=f0, nph=N0, gT=a, gNT=b, dt=dt, steps=n, ce=ce)
    _run(driver, tmp_path, "coupled_adjoint", fill="random:6")
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64
    assert nerr(_out(tmp_path, "gN", rN.shape), rN) <= TOL64
    assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64


@pytest.mark.parametrize("dtype,order", [("f64", 1), ("f32", 1), ("f64", 2), ("f32", 2)])
def test_pair_records_with_rounded_up_mode_count(driver, tmp_path, dtype, order):
    """Five modes: the pair-record kernels run with their mode-slot count
    rounded up to six, the sixth slot re-reading the fifth and counting as
    empty.  Forward and reverse (dL/df, dL/d|g|^2) against the oracle, with
    the {hw, N} table in either order."""
    s = synth.tb_system(kn=24, qn=12, target_states=300, einstein_eV=(0.02, 0.05))
    assert s.n_modes == 5
    f = 0.05 + 0.9 * synth.random_occupations(s, 101)
    nph = s.nph(300.0)
    lam = np.random.default_rng(102).normal(size=s.n_states)
    _write(tmp_path, s, dtype, f=f, lam=lam, nph=nph, B=1, layout=3, table_order=order)
    _run(driver, tmp_path, "forward", fill="random:7")
    _run(driver, tmp_path, "vjp", fill="random:8")
    r = s if dtype == "f64" else _round32(s)
    if dtype == "f32":
        f, nph, lam = (x.astype(np.float32).astype(np.float64) for x in (f, nph, lam))
    tol = TOL64 if dtype == "f64" else TOL32
    ref = oracle.collision(r, f, nph)
    if dtype == "f64":
        assert nerr(_out(tmp_path, "I"), ref) <= tol
    else:
        rin, rout = oracle.collision_inout(r, f, nph)
        scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
        assert np.abs(_out(tmp_path, "I") - ref).max() / scale <= tol
    rf, rg = oracle.collision_vjp(r, f, nph, lam)
    assert nerr(_out(tmp_path, "gf"), rf) <= tol
    assert nerr(_out(tmp_path, "gg2"), rg) <= tol


@pytest.mark.parametrize("window,threads,order,rows", [(64, 256, 1, 1), (200, 512, 1, 1), (1000, 768, 1, 4),
                                                      (64, 256, 2, 1), (1000, 1024, 2, 1), (0, 1024, 1, 64)])
def test_pair_windows_and_workgroup_sizes(driver, tmp_path, window, threads, order, rows):
    """Pair-record passes with smaller LDS windows (more tiles, some on the
    global partner-side accumulator), other workgroup sizes, and the records
    of the LDS tiles in q order (1) or destination order (2): forward and
    reverse against the oracle under a random fill of fresh memory."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    f = synth.random_occupations(s, 131)
    lam = np.random.default_rng(132).normal(size=s.n_states)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f, lam=lam, nph=nph, B=1, layout=3, pair_window=window, pair_threads=threads,
           pair_order=order, pair_rows=rows)
    _run(driver, tmp_path, "forward", fill="random:%d" % window)
    assert nerr(_out(tmp_path, "I"), oracle.collision(s, f, nph)) <= TOL64
    _run(driver, tmp_path, "vjp", fill="random:%d" % threads)
    rf, rg = oracle.collision_vjp(s, f, nph, lam)
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64
    assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64


def test_tuning_rejects_out_of_range_knobs(driver, tmp_path):
    """Record order, row groups, workgroup size, window and table order out
    of range: each set_tuning call fails with INVALID_ARGUMENT and leaves the
    plan's q-ordered pair pass working."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    f = synth.random_occupations(s, 151)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f, nph=nph, B=1, layout=3)
    _run(driver, tmp_path, "tuning_rejects")
    assert _out(tmp_path, "status").tolist() == [1.0] * 8   # EPHBTE_INVALID_ARGUMENT
    assert nerr(_out(tmp_path, "I"), oracle.collision(s, f, nph)) <= TOL64


@pytest.mark.parametrize("layout,fill,order,porder", [(3, "random:9", 1, 1), (2, None, 1, 1), (3, "random:10", 2, 1),
                                                       (3, "random:11", 1, 2)])
def test_vjp_six_modes(driver, tmp_path, layout, fill, order, porder):
    """Reverse pass on the six-mode tight-binding system: over pair records
    (whose consecutive channels are written as 16-byte pairs; records in q or
    destination order) and over entries; every |g|^2 gradient is overwritten
    (the buffer starts at 0.5)."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    f = synth.random_occupations(s, 111)
    lam = np.random.default_rng(112).normal(size=s.n_states)
    nph = s.nph(300.0)
    _write(tmp_path, s, f=f, lam=lam, nph=nph, B=1, layout=layout, gg2_fill=0.5, table_order=order,
           pair_order=porder)
    _run(driver, tmp_path, "vjp", fill=fill)
    rf, rg = oracle.collision_vjp(s, f, nph, lam)
    assert nerr(_out(tmp_path, "gf"), rf) <= TOL64
    assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64


BOSE_CASES = [("forward", dict(B=1, layout=3)), ("forward", dict(B=1, layout=2)), ("forward", dict(B=1, layout=1)),
              ("forward", dict(B=9)), ("forward", dict(B=3, nph_per_batch=1)), ("forward", dict(B=9, nph_per_batch=1)),
              ("vjp", dict(B=1, layout=3)), ("vjp", dict(B=1, layout=1)), ("vjp", dict(B=9)),
              ("vjp_nph", dict()), ("rt", dict(B=1, dt=200.0, steps=2)),
              ("adjoint", dict(dt=200.0, steps=3, ce=2))]


@pytest.mark.parametrize("k", range(len(BOSE_CASES)))
def test_bose_plan(driver, tmp_path, k):
    """Phonon-phonon scattering on a Bose plan (statistics = 1): every entry
    point it serves against the oracle's Bose integral, under random fills of
    fresh memory: forward over the three layouts, batched and with a bath per
    vector; reverse (dL/dn, dL/d|V|^2) at B = 1 and batched; dL/dN; RK4 steps
    and their adjoint."""
    mode, kw = BOSE_CASES[k]
    s = synth.ph_ph_system(n=4)
    B = kw.get("B", 1)
    rng = np.random.default_rng(40 + k)
    F = np.stack([synth.bose_occupations(s, 300.0, seed=50 + b) for b in range(B)])
    lam = rng.normal(size=(B, s.n_states))
    per = kw.get("nph_per_batch", 0)
    tabs = [synth.bose_einstein(s.hw, 250.0 + 30.0 * b) for b in range(B if per else 1)]
    nph = np.stack(tabs) if per else tabs[0]
    gT = rng.normal(size=s.n_states)
    _write(tmp_path, s, f=F, lam=lam, nph=nph, gT=gT, statistics=1, **kw)
    _run(driver, tmp_path, mode, fill="random:%d" % (60 + k))
    if mode == "forward":
        got = _out(tmp_path, "I", (B, s.n_states))
        for b in range(B):
            ref = oracle.collision_bose(s, F[b], tabs[b if per else 0])
            assert nerr(got[b], ref) <= TOL64, b
    elif mode == "vjp":
        gf = _out(tmp_path, "gf", (B, s.n_states))
        rg = 0
        for b in range(B):
            rn, rg_b, _ = oracle.collision_bose_vjp(s, F[b], nph, lam[b])
            assert nerr(gf[b], rn) <= TOL64, b
            rg = rg + rg_b
        assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64
    elif mode == "vjp_nph":
        _, _, rN = oracle.collision_bose_vjp(s, F[0], nph, lam[0])
        assert nerr(_out(tmp_path, "gN", rN.shape), rN) <= TOL64
    elif mode == "rt":
        ref = F[0]
        for _ in range(kw["steps"]):
            ref = oracle.rk4_step(s, ref, nph, kw["dt"], statistics="bose")
        # the increment over the steps carries the bar
        for name in ("f", "f_graph"):
            assert nerr(_out(tmp_path, name) - F[0], ref - F[0]) <= TOL64, name
    else:
        _, rn, rg = oracle.rk4_trajectory_grad(s, F[0], nph, kw["dt"], kw["steps"], gT, statistics="bose")
        assert nerr(_out(tmp_path, "gf"), rn) <= TOL64
        assert nerr(_out(tmp_path, "gg2"), rg) <= TOL64


def test_bose_plan_fp32_and_rejections(driver, tmp_path):
    """FP32 Bose forward pass over pair records against the oracle on
    FP32-rounded inputs, and the entry points defined for Fermi statistics
    only (allocation-free pass, phonon-side rate, coupled step, field term,
    transport) return INVALID_ARGUMENT on a Bose plan."""
    s = synth.ph_ph_system(n=4)
    n = synth.bose_occupations(s, 300.0, seed=70)
    nph = synth.bose_einstein(s.hw, 300.0)
    _write(tmp_path, s, "f32", f=n, nph=nph, B=1, layout=3, statistics=1)
    _run(driver, tmp_path, "forward")
    r = _round32(s)
    n32, N32 = n.astype(np.float32).astype(np.float64), nph.astype(np.float32).astype(np.float64)
    assert nerr(_out(tmp_path, "I"), oracle.collision_bose(r, n32, N32)) <= TOL32
    _write(tmp_path, s, f=n, nph=nph, B=1, statistics=1)
    _run(driver, tmp_path, "bose_rejects")
    assert _out(tmp_path, "status").tolist() == [1.0] * 5   # EPHBTE_INVALID_ARGUMENT
