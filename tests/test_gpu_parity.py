"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Error metric: normwise, err = max_s |I_gpu - I_ref| / max_s |I_ref|.  For
FP32 the reference is the FP64 oracle on the FP32-rounded inputs, and the
norm is max(max|I_ref|, 1e-2 max(in, out)) so that near-equilibrium vectors
(in and out rates cancelling) are judged against their gross rates.
Bars: 1e-10 (FP64, FP64 accumulation), 1e-5 (FP32, FP32 accumulation).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2511_03683_amd as lib
    return lib


def say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def nerr(x, ref, scale=None):
    s = np.abs(ref).max() if scale is None else scale
    err = float(np.abs(np.asarray(x) - ref).max() / max(s, 1e-300))
    print(f"[gpu-err] {err:.3e}", flush=True)
    return err


def rate_bound(sys, nph):
    """Per-state bound on |I_d| that holds for any f in [0, 1]: every channel
    of d adds at most C |g|^2 (2 N_max + 1) / (sigma sqrt(2 pi)) in magnitude
    (C = 2 pi / (hbar N_q); each Gaussian is at most its peak)."""
    C = 2 * np.pi / (oracle.HBAR_EV_FS * sys.n_q_norm) / (sys.sigma * np.sqrt(2 * np.pi))
    w = np.asarray(sys.g2, np.float64) * (2 * np.abs(nph).max() + 1) * C
    S = sys.n_states
    return (np.bincount(sys.ch_i, weights=w, minlength=S) + np.bincount(sys.ch_j, weights=w, minlength=S))


def plausible(x, bound):
    """Every unsampled output is finite and within the per-state bound."""
    x = np.asarray(x)
    assert np.isfinite(x).all()
    assert np.all(np.abs(x) <= bound * (1 + 1e-6) + 1e-300)


def incident(sys, rows):
    """Keep mask of the channels that touch the given states."""
    return np.isin(sys.ch_i, rows) | np.isin(sys.ch_j, rows)


def gross_scale(sys, f, nph, ref, rows=None):
    """Norm of the FP32 bar: max(max|I_ref|, 1e-2 max(in, out)) over the rows
    compared, from the oracle (in - out = I)."""
    rin, rout = oracle.collision_inout(sys, f, nph)
    if rows is not None:
        rin, rout, ref = rin[rows], rout[rows], ref[rows]
    return max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))


def round32(s):
    """Copy of a system with every floating input rounded to FP32."""
    import copy
    r = copy.copy(s)
    r.eps = s.eps.astype(np.float32).astype(np.float64)
    r.hw = s.hw.astype(np.float32).astype(np.float64)
    r.g2 = s.g2.astype(np.float32).astype(np.float64)
    return r


def run_I(E, s, f, nph, dtype="f64", tuning=None):
    plan = E.build_channels(s, dtype=dtype, device=0)
    if tuning:
        E.set_tuning(plan, **tuning)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    out = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    plan.close()
    return out


SYSTEMS = {
    "parabolic8_c1occ": (lambda: synth.parabolic_system(8), lambda s: synth.c1_occupations(s)),
    "parabolic8_random": (lambda: synth.parabolic_system(8), lambda s: synth.random_occupations(s, 3)),
    "multiband": (lambda: synth.multiband_system(), lambda s: synth.random_occupations(s, 4)),
    "random_order": (lambda: synth.random_channel_system(n_states=60, n_channels=900, seed=3),
                     lambda s: synth.random_occupations(s, 5)),
    "tb24": (lambda: synth.tb_system(kn=24, qn=12, target_states=400),
             lambda s: synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.9 + 0.2 * synth.random_occupations(s, 6))),
}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_fp64_matches_oracle(E, name):
    mk, occ = SYSTEMS[name]
    s = mk()
    f = np.clip(occ(s), 0, 1)
    nph = s.nph(300.0)
    say(f"fp64 collision {name} S={s.n_states} Nch={s.n_channels}")
    I = run_I(E, s, f, nph)
    ref = oracle.collision(s, f, nph)
    assert nerr(I, ref) <= TOL64


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_fp32_matches_oracle_on_rounded_inputs(E, name):
    mk, occ = SYSTEMS[name]
    s = mk()
    f = np.clip(occ(s), 0, 1).astype(np.float32).astype(np.float64)
    nph = s.nph(300.0).astype(np.float32).astype(np.float64)
    say(f"fp32 collision {name} S={s.n_states} Nch={s.n_channels}")
    I = run_I(E, s, f, nph, dtype="f32")
    r = round32(s)
    ref = oracle.collision(r, f, nph)
    rin, rout = oracle.collision_inout(r, f, nph)
    scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
    assert nerr(I, ref, scale) <= TOL32


@pytest.mark.parametrize("tuning", [dict(chunk_entries=64), dict(chunk_entries=100, block_threads=64),
                                    dict(chunk_entries=300, tile_entries=1000),
                                    dict(chunk_entries=65536, tile_entries=-1),
                                    dict(chunk_entries=1000, block_threads=512),
                                    dict(block_threads=128, xcd_map=2), dict(chunk_entries=7, xcd_map=1)])
def test_split_segments_and_launch_shapes(E, tuning):
    """Segments split over several workgroups (two-level reduction), other
    block sizes and both chunk orders give the oracle's result."""
    s = synth.parabolic_system(8)
    f = synth.random_occupations(s, 9)
    nph = s.nph(300.0)
    say(f"fp64 collision tuning={tuning}")
    I = run_I(E, s, f, nph, tuning=tuning)
    assert nerr(I, oracle.collision(s, f, nph)) <= TOL64


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", ["parabolic8_random", "multiband", "random_order", "tb24"])
def test_single_copy_and_duplicated_layouts(E, name, dtype):
    """The B = 1 forward pass in every layout (each channel evaluated in both of
    its rows; once with fixed-point partner sums, one entry per channel; once
    over pair records, where the plan has them) against the oracle; each
    result is bitwise reproducible, also with rows split in chunks."""
    mk, occ = SYSTEMS[name]
    s = mk()
    f = np.clip(occ(s), 0, 1)
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    r = s
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
        r = round32(s)
    ref = oracle.collision(r, f, nph)
    if dtype == "f64":
        tol, scale = TOL64, None
    else:
        rin, rout = oracle.collision_inout(r, f, nph)
        tol, scale = TOL32, max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"layouts {dtype} {name}")
    got = {}
    cases = [(1, -1, 0), (2, -1, 0), (2, 37, 0), (1, 37, 0)]
    if E.plan_info(plan)["pair_records"] > 0:
        cases += [(3, -1, 1), (3, 5, 1), (3, -1, 2)]
    for layout, chunk, fexp in cases:
        E.set_tuning(plan, layout=layout, chunk_entries=65536 if chunk < 0 else chunk, fp64_exp=fexp)
        a = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
        b = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
        assert np.array_equal(a, b), (layout, chunk, fexp)
        assert nerr(a, ref, scale) <= tol, (layout, chunk, fexp)
        got[(layout, chunk, fexp)] = a
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pair_pass_shapes_and_table_order(E, dtype):
    """The pair-record passes with smaller LDS windows and other workgroup
    sizes, with the {hw, N} table one block per mode, and with the records of
    the LDS tiles in q order or destination order (switched back and forth on
    one plan): forward and reverse against the oracle; the forward repeats
    bitwise, and in destination order it is bitwise the same for every shape
    (its row sums do not depend on the tiles)."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    f = np.clip(synth.random_occupations(s, 141), 0, 1)
    lam = np.random.default_rng(142).normal(size=s.n_states)
    nph = s.nph(300.0)
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f, lam, nph = (a.astype(np.float32).astype(np.float64) for a in (f, lam, nph))
        r, tdt, tol = round32(s), torch.float32, TOL32
    ref = oracle.collision(r, f, nph)
    rin, rout = oracle.collision_inout(r, f, nph)
    scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
    rf, rg = oracle.collision_vjp(r, f, nph, lam)
    plan = E.build_channels(s, dtype=dtype, device=0)
    assert E.plan_info(plan)["layout"] == 3
    say(f"pair pass shapes {dtype}")
    base = None
    for w, th, order, po, rows in ((0, 0, 1, 1, 0), (64, 256, 1, 1, 0), (500, 512, 1, 1, 16), (1000, 768, 2, 1, 1),
                                   (0, 1024, 2, 2, 0), (64, 256, 1, 2, 0), (500, 512, 2, 2, 0),
                                   (3072 if dtype == "f64" else 4096, 1024, 1, 1, 64)):
        case = (w, th, order, po, rows)
        E.set_tuning(plan, pair_window=w, pair_threads=th, table_order=order, pair_order=po, pair_rows=rows)
        I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
        assert nerr(I, ref, scale) <= tol, case
        assert np.array_equal(I, host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))), case
        if po == 2:
            if base is None:
                base = I
            assert np.array_equal(I, base), case
        gf, gg = E.collision_vjp(plan, dev(f, tdt), dev(nph, tdt), dev(lam, tdt), gg2=True)
        assert nerr(host(gf), rf) <= tol, case
        assert nerr(host(gg), rg) <= tol, case
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_copy_scale_adapts(E, dtype):
    """The single-copy pass's fixed-point scale follows the inputs: |g|^2 scaled
    by 1e6 and 1e-6, phonon occupations of a 3000 K bath, and |g|^2 replaced
    through update_g2 (its per-state bound is recomputed) all match the oracle."""
    s0 = synth.multiband_system()
    f = synth.random_occupations(s0, 31)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    for scale, T in ((1e6, 300.0), (1e-6, 300.0), (1.0, 3000.0)):
        import copy
        s = copy.copy(s0)
        s.g2 = s0.g2 * scale
        nph = s.nph(T)
        ff, nn, r = f, nph, s
        if dtype == "f32":
            ff = f.astype(np.float32).astype(np.float64)
            nn = nph.astype(np.float32).astype(np.float64)
            r = round32(s)
        ref = oracle.collision(r, ff, nn)
        plan = E.build_channels(s, dtype=dtype, device=0)
        say(f"single-copy scale {dtype} g2 x {scale:g}, {T} K")
        got = host(E.collision_integral(plan, dev(ff, tdt), dev(nn, tdt)))
        if dtype == "f64":
            assert nerr(got, ref) <= TOL64, (scale, T)
        else:
            rin, rout = oracle.collision_inout(r, ff, nn)
            assert nerr(got, ref, max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))) <= TOL32
        if scale == 1.0:
            # |g|^2 x 1e3 through update_g2
            s2 = copy.copy(s)
            s2.g2 = s.g2 * 1e3
            E.update_g2(plan, dev(s2.g2))
            r2 = s2 if dtype == "f64" else round32(s2)
            ref2 = oracle.collision(r2, ff, nn)
            got2 = host(E.collision_integral(plan, dev(ff, tdt), dev(nn, tdt)))
            if dtype == "f64":
                assert nerr(got2, ref2) <= TOL64
            else:
                rin, rout = oracle.collision_inout(r2, ff, nn)
                assert nerr(got2, ref2, max(np.abs(ref2).max(), 1e-2 * max(rin.max(), rout.max()))) <= TOL32
        plan.close()


def test_deterministic_and_batched_columns(E):
    s = synth.multiband_system()
    nph = dev(s.nph(300.0))
    plan = E.build_channels(s, device=0)
    # B = 3 runs the per-row pass; its columns equal B = 1 bitwise in that layout
    E.set_tuning(plan, layout=1)
    F = np.stack([synth.random_occupations(s, k) for k in range(3)])
    say("determinism + strided batch")
    I1 = host(E.collision_integral(plan, dev(F[0]), nph))
    I1b = host(E.collision_integral(plan, dev(F[0]), nph))
    assert np.array_equal(I1, I1b), "bitwise reproducible"
    big = torch.zeros((3, s.n_states + 5), dtype=torch.float64, device="cuda:0")
    big[:, :s.n_states] = dev(F)
    Fv = big[:, :s.n_states]
    out = torch.full((3, s.n_states + 3), 7.0, dtype=torch.float64, device="cuda:0")
    E.collision_integral(plan, Fv, nph, out=out[:, :s.n_states])
    got = host(out)
    for b in range(3):
        ref_b = host(E.collision_integral(plan, dev(F[b]), nph))
        assert np.array_equal(got[b, :s.n_states], ref_b)
        assert np.all(got[b, s.n_states:] == 7.0), "padding untouched"
    plan.close()


BATCH_SYSTEMS = {
    "tb24": lambda: synth.tb_system(kn=24, qn=12, target_states=400),
    "multiband": lambda: synth.multiband_system(),
    "random_order": lambda: synth.random_channel_system(n_states=60, n_channels=900, seed=3),
    "parabolic8": lambda: synth.parabolic_system(8),
}


@pytest.mark.parametrize("B,dtype,name", [(8, "f64", "tb24"), (64, "f64", "tb24"), (70, "f64", "tb24"),
                                          (64, "f32", "tb24"), (9, "f64", "multiband"),
                                          (64, "f64", "random_order"), (64, "f64", "parabolic8"),
                                          (65, "f32", "parabolic8")])
def test_batched_pass_matches_oracle(E, B, dtype, name):
    """B vectors in one pass (coefficients evaluated once per entry and applied
    to every vector), strided input/output, every column against the oracle."""
    s = BATCH_SYSTEMS[name]()
    rng = np.random.default_rng(B)
    F = rng.uniform(size=(B, s.n_states))
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        F = F.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"batched {dtype} B={B} {name} S={s.n_states}")
    big = torch.zeros((B, s.n_states + 3), dtype=tdt, device="cuda:0")
    big[:, :s.n_states] = dev(F, tdt)
    out = torch.full((B, s.n_states + 1), 5.0, dtype=tdt, device="cuda:0")
    E.collision_integral(plan, big[:, :s.n_states], dev(nph, tdt), out=out[:, :s.n_states])
    got = host(out)
    assert np.all(got[:, s.n_states:] == 5.0)
    r = s if dtype == "f64" else round32(s)
    for b in sorted({0, 1, B // 2, B - 1}):
        ref = oracle.collision(r, F[b], nph)
        if dtype == "f64":
            assert nerr(got[b, :s.n_states], ref) <= TOL64, b
        else:
            rin, rout = oracle.collision_inout(r, F[b], nph)
            scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
            assert nerr(got[b, :s.n_states], ref, scale) <= TOL32, b
    plan.close()


@pytest.mark.parametrize("pt", [16, 48, 160])
def test_batch_partner_tiles(E, pt):
    """Other partner sub-tile sizes of the batched pass (tile shapes from the
    host, sub-tile entry offsets searched on the device) against the oracle."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    B = 16
    F = np.random.default_rng(pt).uniform(size=(B, s.n_states))
    nph = s.nph(300.0)
    plan = E.build_channels(s, device=0)
    say(f"batch partner sub-tile {pt}")
    try:
        E.set_tuning(plan, batch_partners=pt)
    except E.EphbteError as e:
        plan.close()
        assert "LDS" in str(e)
        pytest.skip(f"sub-tile of {pt} partners exceeds this device's LDS per workgroup")
    got = host(E.collision_integral(plan, dev(F), dev(nph)))
    for b in (0, 7, B - 1):
        assert nerr(got[b], oracle.collision(s, F[b], nph)) <= TOL64, b
    plan.close()


def test_autotune_keeps_results(E):
    """The autotuner's choice (single-vector chunking, then the batched
    sub-tile size) leaves the results at the oracle's."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    nph = s.nph(300.0)
    plan = E.build_channels(s, device=0)
    say("autotune B=1 and B=16")
    t1 = E.autotune(plan, 1)
    assert t1["chunk_entries"] in (8192, 16384, 32768, 65536) and t1["block_threads"] in (256, 512)
    assert t1["tile_entries"] == -1 or t1["tile_entries"] > 0
    f = synth.random_occupations(s, 21)
    assert nerr(host(E.collision_integral(plan, dev(f), dev(nph))), oracle.collision(s, f, nph)) <= TOL64
    t16 = E.autotune(plan, 16)
    assert t16["batch_partners"] in (48, 64, 96, 128, 160)
    F = np.random.default_rng(16).uniform(size=(16, s.n_states))
    got = host(E.collision_integral(plan, dev(F), dev(nph)))
    for b in (0, 15):
        assert nerr(got[b], oracle.collision(s, F[b], nph)) <= TOL64, b
    plan.close()


def test_autotune_cache(E, tmp_path):
    """A cached tuning is applied without timing (a hand-edited entry comes
    back as written and the results stay at the oracle's); single and batched
    entries live side by side; a file that is not a cache is refused and left
    as it was."""
    import json
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    nph = s.nph(300.0)
    path = str(tmp_path / "tune.json")
    plan = E.build_channels(s, device=0)
    say("autotune cache")
    t1 = E.autotune(plan, 1, cache_path=path)
    t16 = E.autotune(plan, 16, cache_path=path)
    c = json.load(open(path))
    assert len(c) == 2
    single = [k for k in c if k.endswith("|single")][0]
    batched = [k for k in c if k.endswith("|batched")][0]
    assert c[single]["chunk_entries"] == t1["chunk_entries"]
    assert c[batched]["batch_partners"] == t16["batch_partners"]
    c[single] = {"block_threads": 128, "chunk_entries": 4096, "tile_entries": -1}
    c[batched] = {"batch_partners": 64 if t16["batch_partners"] != 64 else 48}
    json.dump(c, open(path, "w"))
    plan2 = E.build_channels(s, device=0)
    u1 = E.autotune(plan2, 1, cache_path=path)
    assert (u1["block_threads"], u1["chunk_entries"]) == (128, 4096)
    u16 = E.autotune(plan2, 16, cache_path=path)
    assert u16["batch_partners"] == c[batched]["batch_partners"]
    assert json.load(open(path)) == c, "a hit leaves the file as it was"
    f = synth.random_occupations(s, 22)
    assert nerr(host(E.collision_integral(plan2, dev(f), dev(nph))), oracle.collision(s, f, nph)) <= TOL64
    F = np.random.default_rng(17).uniform(size=(16, s.n_states))
    got = host(E.collision_integral(plan2, dev(F), dev(nph)))
    assert nerr(got[3], oracle.collision(s, F[3], nph)) <= TOL64
    bad = tmp_path / "other.json"
    bad.write_text('{"something": [1, 2, 3]}')
    with pytest.raises(E.EphbteError, match="autotune cache"):
        E.autotune(plan2, 1, cache_path=str(bad))
    assert bad.read_text() == '{"something": [1, 2, 3]}'
    plan.close()
    plan2.close()


def test_batched_rk4_matches_oracle(E):
    s = synth.multiband_system()
    nph = s.nph(300.0)
    B, dt, n = 12, 0.5, 3
    F = np.stack([synth.random_occupations(s, 40 + b) for b in range(B)])
    plan = E.build_channels(s, device=0)
    say("batched rt_step")
    Ft = dev(F)
    E.rt_step(plan, Ft, dev(nph), dt, n, use_graph=True)
    got = host(Ft)
    for b in (0, 5, B - 1):
        ref = F[b].copy()
        for _ in range(n):
            ref = oracle.rk4_step(s, ref, nph, dt)
        assert nerr(got[b] - F[b], ref - F[b]) <= TOL64
    plan.close()


def test_invariants_on_gpu(E):
    s = synth.parabolic_system(8)
    nph = s.nph(300.0)
    plan = E.build_channels(s, device=0)
    say("invariants: Pauli, particle number")
    for v in (0.0, 1.0):
        I = host(E.collision_integral(plan, dev(np.full(s.n_states, v)), dev(nph)))
        assert np.all(I == 0.0)
    f = synth.random_occupations(s, 12)
    I = host(E.collision_integral(plan, dev(f), dev(nph)))
    assert abs(I.sum()) <= 1e-13 * np.abs(I).sum()
    plan.close()


def test_resonant_ladder_equilibrium_on_gpu(E):
    s = synth.ladder_system()
    nph = s.nph(300.0)
    f_eq = synth.fermi_dirac(s.eps, 0.1, 300.0)
    f_hot = synth.fermi_dirac(s.eps, 0.1, 900.0)
    say("ladder equilibrium")
    I_eq = run_I(E, s, f_eq, nph)
    I_hot = run_I(E, s, f_hot, nph)
    assert np.abs(I_eq).max() <= 1e-13 * np.abs(I_hot).max()


def test_empty_and_isolated(E):
    s = synth.random_channel_system(n_states=10, n_channels=0)
    f = synth.random_occupations(s, 1)
    say("empty channel list")
    assert np.all(run_I(E, s, f, s.nph(300.0)) == 0.0)
    s2 = synth.random_channel_system(n_states=30, n_channels=20, seed=8)
    isolated = np.setdiff1d(np.arange(30), np.concatenate([s2.ch_i, s2.ch_j]))
    assert isolated.size > 0
    f2 = synth.random_occupations(s2, 2)
    I2 = run_I(E, s2, f2, s2.nph(300.0))
    assert np.all(I2[isolated] == 0.0)
    assert nerr(I2, oracle.collision(s2, f2, s2.nph(300.0))) <= TOL64


# ------------------------------------------------------------------ reverse mode
@pytest.mark.parametrize("name", ["multiband", "random_order", "parabolic8_random"])
def test_vjp_matches_oracle(E, name):
    """Reverse pass: overwrite and accumulate of dL/d|g|^2, batched vectors."""
    mk, occ = SYSTEMS[name]
    s = mk()
    f = np.clip(occ(s), 0, 1)
    nph = s.nph(300.0)
    lam = np.random.default_rng(2).normal(size=s.n_states)
    plan = E.build_channels(s, device=0)
    say(f"vjp {name}")
    gf, gg = E.collision_vjp(plan, dev(f), dev(nph), dev(lam), want_f=True, gg2=True)
    rf, rg = oracle.collision_vjp(s, f, nph, lam)
    assert nerr(host(gf), rf) <= TOL64
    assert nerr(host(gg), rg) <= TOL64
    # bitwise reproducible
    gf2, gg2 = E.collision_vjp(plan, dev(f), dev(nph), dev(lam), want_f=True, gg2=True)
    assert np.array_equal(host(gf2), host(gf)) and np.array_equal(host(gg2), host(gg))
    # accumulate adds onto the existing buffer
    E.collision_vjp(plan, dev(f), dev(nph), dev(lam), want_f=False, gg2=gg, accumulate=True)
    assert nerr(host(gg), 2 * rg) <= TOL64
    # batched: dL/dg2 is summed over the vectors
    lam2 = np.random.default_rng(3).normal(size=s.n_states)
    F = np.stack([f, np.clip(occ(s)[::-1].copy(), 0, 1)])
    L = np.stack([lam, lam2])
    gfb, ggb = E.collision_vjp(plan, dev(F), dev(nph), dev(L), gg2=True)
    r0 = oracle.collision_vjp(s, F[0], nph, L[0])
    r1 = oracle.collision_vjp(s, F[1], nph, L[1])
    assert nerr(host(gfb)[1], r1[0]) <= TOL64
    assert nerr(host(ggb), r0[1] + r1[1]) <= TOL64
    plan.close()


def test_vjp_fp32(E):
    s = synth.multiband_system()
    f = synth.random_occupations(s, 4).astype(np.float32).astype(np.float64)
    nph = s.nph(300.0).astype(np.float32).astype(np.float64)
    lam = np.random.default_rng(2).normal(size=s.n_states).astype(np.float32).astype(np.float64)
    plan = E.build_channels(s, dtype="f32", device=0)
    say("vjp fp32")
    gf, gg = E.collision_vjp(plan, dev(f, torch.float32), dev(nph, torch.float32),
                             dev(lam, torch.float32), gg2=True)
    rf, rg = oracle.collision_vjp(round32(s), f, nph, lam)
    assert nerr(host(gf), rf) <= 1e-5
    assert nerr(host(gg), rg) <= 1e-5
    plan.close()


@pytest.mark.parametrize("dtype,B", [("f64", 5), ("f32", 5), ("f64", 20), ("f32", 70)])
def test_bath_per_vector(E, dtype, B):
    """nph [B, Nq, n_modes]: vector b sees the bath of its own temperature,
    forward and reverse (dL/d|g|^2 summed over the vectors); B >= 8 runs the
    forward pass batched, the baths in groups of 64 vectors."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    temps = [[150.0, 300.0, 450.0, 220.0, 600.0][b % 5] + 7.0 * b for b in range(B)]
    F = np.stack([np.clip(synth.random_occupations(s, 20 + b), 0, 1) for b in range(B)])
    NPH = np.stack([s.nph(T) for T in temps])
    L = np.random.default_rng(5).normal(size=(B, s.n_states))
    r = s
    tdt, tol = torch.float64, TOL64
    if dtype == "f32":
        F, NPH, L = (a.astype(np.float32).astype(np.float64) for a in (F, NPH, L))
        r, tdt, tol = round32(s), torch.float32, TOL32
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"bath per vector {dtype} B={B} S={s.n_states} Nch={s.n_channels}")
    I = host(E.collision_integral(plan, dev(F, tdt), dev(NPH, tdt)))
    for b in range(B):
        ref = oracle.collision(r, F[b], NPH[b])
        rin, rout = oracle.collision_inout(r, F[b], NPH[b])
        scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
        assert nerr(I[b], ref, scale) <= tol, b
    # the shared-table call on the same vectors differs from it
    Ish = host(E.collision_integral(plan, dev(F, tdt), dev(NPH[1], tdt)))
    assert np.abs(Ish[0] - I[0]).max() > 1e-3 * np.abs(I[0]).max()
    gf, gg = E.collision_vjp(plan, dev(F, tdt), dev(NPH, tdt), dev(L, tdt), gg2=True)
    gf, gg = host(gf), host(gg)
    rg_sum = 0
    for b in range(B):
        rf, rg = oracle.collision_vjp(r, F[b], NPH[b], L[b])
        assert nerr(gf[b], rf) <= tol, b
        rg_sum = rg_sum + rg
    assert nerr(gg, rg_sum) <= tol
    with pytest.raises(ValueError):
        E.collision_integral(plan, dev(F, tdt), dev(NPH[:2], tdt))
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_channel_selection_at_build(E, dtype):
    """A plan built with the energy and |g|^2 selection computes Eq. 2 over the
    oracle's kept channels; the |g|^2 gradients of removed channels are 0."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    nsig, g2min = 2.5, 5e-4
    keep = oracle.select_channels(s, nsig, g2min)
    sub = oracle.subset(s, keep)
    f = np.clip(synth.random_occupations(s, 31), 0, 1)
    nph = s.nph(300.0)
    lam = np.random.default_rng(8).normal(size=s.n_states)
    r, tdt, tol = sub, torch.float64, TOL64
    if dtype == "f32":
        f, nph, lam = (a.astype(np.float32).astype(np.float64) for a in (f, nph, lam))
        r, tdt, tol = round32(sub), torch.float32, TOL32
    plan = E.build_channels(s, dtype=dtype, device=0, energy_nsigma=nsig, g2_min=g2min)
    say(f"selection at build {dtype} kept {int(keep.sum())} of {s.n_channels}")
    info = E.plan_info(plan)
    assert info["n_channels"] == s.n_channels and info["channels_kept"] == int(keep.sum())
    assert info["entries"] == 2 * int(keep.sum())
    I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    ref = oracle.collision(r, f, nph)
    rin, rout = oracle.collision_inout(r, f, nph)
    scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
    assert nerr(I, ref, scale) <= tol
    gg = torch.full((s.n_channels,), 7.0, dtype=torch.float64, device="cuda:0")
    gf, gg = E.collision_vjp(plan, dev(f, tdt), dev(nph, tdt), dev(lam, tdt), gg2=gg)
    rf, rg = oracle.collision_vjp(r, f, nph, lam)
    gg = host(gg)
    assert np.all(gg[~keep] == 0.0)
    assert nerr(gg[keep], rg) <= tol
    assert nerr(host(gf), rf) <= tol
    plan.close()


@pytest.mark.parametrize("dtype,B", [("f64", 8), ("f64", 70), ("f32", 64), ("f32", 9)])
def test_batched_vjp(E, dtype, B):
    """B >= 8 vectors sharing one bath in one reverse pass per 64 vectors:
    dL/df per column and dL/d|g|^2 summed over the columns match the oracle;
    overwrite, accumulate, gradient-only and strided (ld > S) forms; repeat
    calls are bitwise equal."""
    s = synth.tb_system(kn=24, qn=12, target_states=400)
    S = s.n_states
    rng = np.random.default_rng(40 + B)
    F = np.clip(rng.uniform(0, 1, size=(B, S)), 0, 1)
    L = rng.normal(size=(B, S))
    nph = s.nph(300.0)
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        F, L, nph = (a.astype(np.float32).astype(np.float64) for a in (F, L, nph))
        r, tdt, tol = round32(s), torch.float32, TOL32
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"batched vjp {dtype} B={B} S={S} Nch={s.n_channels}")
    # strided operands: rows of a wider buffer
    Fw = torch.zeros((B, S + 13), dtype=tdt, device="cuda:0")
    Fw[:, :S] = dev(F, tdt)
    Lw = torch.zeros((B, S + 5), dtype=tdt, device="cuda:0")
    Lw[:, :S] = dev(L, tdt)
    gf, gg = E.collision_vjp(plan, Fw[:, :S], dev(nph, tdt), Lw[:, :S], gg2=True)
    gf, gg = host(gf), host(gg)
    rg_sum = 0
    for b in range(B):
        rf, rg = oracle.collision_vjp(r, F[b], nph, L[b])
        assert nerr(gf[b], rf) <= tol, b
        rg_sum = rg_sum + rg
    assert nerr(gg, rg_sum) <= tol
    gf2, gg2 = E.collision_vjp(plan, dev(F, tdt), dev(nph, tdt), dev(L, tdt), gg2=True)
    assert np.array_equal(host(gf2), gf) and np.array_equal(host(gg2), gg)
    acc = torch.full((s.n_channels,), 0.25, dtype=torch.float64, device="cuda:0")
    none, acc = E.collision_vjp(plan, dev(F, tdt), dev(nph, tdt), dev(L, tdt), want_f=False,
                                gg2=acc, accumulate=True)
    assert none is None
    assert nerr(host(acc) - 0.25, rg_sum) <= tol
    gf3, _ = E.collision_vjp(plan, dev(F, tdt), dev(nph, tdt), dev(L, tdt))
    assert np.array_equal(host(gf3), gf)
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_elastic_mechanism(E, dtype):
    """A defect mechanism flagged elastic (hw = 0, N = 0) beside three phonon
    modes: forward and reverse passes match Eq. 2 in the oracle, and the
    elastic part alone matches the oracle's elastic golden rule."""
    s = synth.defect_system(6, with_phonons=True)
    e = s.meta["elastic_mode"]
    f = synth.random_occupations(s, 14)
    nph = s.nph(300.0)
    lam = np.random.default_rng(9).normal(size=s.n_states)
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f, nph, lam = (a.astype(np.float32).astype(np.float64) for a in (f, nph, lam))
        r, tdt, tol = round32(s), torch.float32, TOL32
    say(f"elastic mechanism {dtype} S={s.n_states} Nch={s.n_channels}")
    plan = E.build_channels(s, dtype=dtype, device=0, elastic_modes=1 << e)
    I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    ref = oracle.collision(r, f, nph)
    rin, rout = oracle.collision_inout(r, f, nph)
    scale = max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))
    assert nerr(I, ref, scale) <= tol
    gf, gg = E.collision_vjp(plan, dev(f, tdt), dev(nph, tdt), dev(lam, tdt), gg2=True)
    rf, rg = oracle.collision_vjp(r, f, nph, lam)
    assert nerr(host(gf), rf) <= tol and nerr(host(gg), rg) <= tol
    plan.close()
    el = oracle.subset(s, np.asarray(s.ch_nu) == e)
    plan = E.build_channels(el, dtype=dtype, device=0, elastic_modes=1 << e)
    I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    ref = oracle.collision_elastic(round32(el) if dtype == "f32" else el, f)
    assert nerr(I, ref) <= tol
    plan.close()


PH_SYSTEMS = {
    "multiband": lambda: synth.multiband_system(),
    "tb24": lambda: synth.tb_system(kn=24, qn=12, target_states=400),
    "parabolic8": lambda: synth.parabolic_system(8),
}


@pytest.mark.parametrize("name,dtype", [(n, d) for n in PH_SYSTEMS for d in ("f64", "f32")])
def test_phonon_rate_matches_oracle(E, name, dtype):
    """dN/dt of every (q, mode) against the oracle; bitwise repeatable; the
    bins are cleared between calls; update_g2 rescales it."""
    s = PH_SYSTEMS[name]()
    f = synth.random_occupations(s, 50)
    nph = s.nph(300.0)
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f, nph = f.astype(np.float32).astype(np.float64), nph.astype(np.float32).astype(np.float64)
        r, tdt, tol = round32(s), torch.float32, TOL32
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"phonon rate {name} {dtype} S={s.n_states} Nch={s.n_channels}")
    got = host(E.phonon_rate(plan, dev(f, tdt), dev(nph, tdt)))
    ref = oracle.phonon_rate(r, f, nph)
    assert np.abs(ref).max() > 0
    assert nerr(got, ref) <= tol
    again = host(E.phonon_rate(plan, dev(f, tdt), dev(nph, tdt)))
    assert np.array_equal(again, got)
    E.update_g2(plan, dev(3.0 * s.g2))
    tri = host(E.phonon_rate(plan, dev(f, tdt), dev(nph, tdt)))
    assert nerr(tri, 3.0 * ref) <= tol
    plan.close()


def test_phonon_rate_skips_elastic_mechanisms(E):
    s = synth.defect_system(6, with_phonons=True)
    e = s.meta["elastic_mode"]
    f = synth.random_occupations(s, 51)
    nph = s.nph(300.0)
    plan = E.build_channels(s, device=0, elastic_modes=1 << e)
    say("phonon rate with an elastic mechanism")
    got = host(E.phonon_rate(plan, dev(f), dev(nph)))
    ref = oracle.phonon_rate(oracle.subset(s, np.asarray(s.ch_nu) != e), f, nph)
    assert np.all(got[:, e] == 0.0)
    assert nerr(got, ref) <= TOL64
    plan.close()


@pytest.mark.parametrize("name,dtype", [("multiband", "f64"), ("tb24", "f64"), ("multiband", "f32")])
def test_rt_step_coupled_matches_oracle(E, name, dtype):
    """Electrons and phonons stepped together against the oracle's coupled
    RK4; N stays even in q."""
    s = PH_SYSTEMS[name]()
    f0 = 0.1 + 0.8 * synth.random_occupations(s, 52)
    N0 = s.nph(300.0) * 1.5
    dt, n = 1.0, 3
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f0, N0 = f0.astype(np.float32).astype(np.float64), N0.astype(np.float32).astype(np.float64)
        r, tdt, tol = round32(s), torch.float32, 1e-5
    rf, rN = f0, N0
    for _ in range(n):
        rf, rN = oracle.rk4_coupled_step(r, rf, rN, dt)
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"coupled rt step {name} {dtype} S={s.n_states} Nch={s.n_channels}")
    ft, Nt = dev(f0, tdt), dev(N0, tdt)
    E.rt_step_coupled(plan, ft, Nt, dt, n)
    gf, gN = host(ft), host(Nt)
    assert np.abs(rN - N0).max() > 0
    assert nerr(gf - f0, rf - f0) <= tol
    assert nerr(gN - N0, rN - N0) <= tol
    assert np.array_equal(oracle.even_in_q(s, gN), gN) or np.abs(oracle.even_in_q(s, gN) - gN).max() <= 1e-15 * np.abs(gN).max()
    plan.close()


def _uneven_bath(s, seed):
    """A positive phonon table that is not even in q: a q / -q mix-up in a
    reverse mode changes the result."""
    return s.nph(300.0) * np.random.default_rng(seed).uniform(0.5, 1.5, size=s.hw.shape)


@pytest.mark.parametrize("name,dtype", [("multiband", "f64"), ("tb24", "f64"), ("multiband", "f32")])
def test_collision_vjp_nph_matches_oracle(E, name, dtype):
    s = PH_SYSTEMS[name]()
    f = synth.random_occupations(s, 61)
    N = _uneven_bath(s, 62)
    lam = np.random.default_rng(63).normal(size=s.n_states)
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f, N, lam = (x.astype(np.float32).astype(np.float64) for x in (f, N, lam))
        r, tdt, tol = round32(s), torch.float32, TOL32
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"collision vjp nph {name} {dtype}")
    got = host(E.collision_vjp_nph(plan, dev(f, tdt), dev(N, tdt), dev(lam, tdt)))
    plan.close()
    assert nerr(got, oracle.collision_vjp_nph(r, f, N, lam)) <= tol


@pytest.mark.parametrize("name,dtype", [("multiband", "f64"), ("tb24", "f64"), ("multiband", "f32")])
def test_phonon_rate_vjp_matches_oracle(E, name, dtype):
    s = PH_SYSTEMS[name]()
    f = synth.random_occupations(s, 71)
    N = _uneven_bath(s, 72)
    mu = np.random.default_rng(73).normal(size=N.shape)
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f, N, mu = (x.astype(np.float32).astype(np.float64) for x in (f, N, mu))
        r, tdt, tol = round32(s), torch.float32, TOL32
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"phonon rate vjp {name} {dtype}")
    gf, gN, gg = E.phonon_rate_vjp(plan, dev(f, tdt), dev(N, tdt), dev(mu, tdt), gg2=True)
    plan.close()
    rf, rN, rg = oracle.phonon_rate_vjp(r, f, N, mu)
    assert nerr(host(gf), rf) <= tol
    assert nerr(host(gN), rN) <= tol
    assert nerr(host(gg), rg) <= tol


@pytest.mark.parametrize("name,dtype,ce", [("multiband", "f64", 1), ("multiband", "f64", 2), ("tb24", "f64", 3),
                                           ("multiband", "f32", 2)])
def test_rt_adjoint_coupled_matches_oracle(E, name, dtype, ce):
    """Gradients with respect to f0, N0 and |g|^2 through three coupled RK4
    steps against the oracle's discrete adjoint with every stage stored."""
    s = PH_SYSTEMS[name]()
    f0 = 0.1 + 0.8 * synth.random_occupations(s, 81)
    N0 = s.nph(300.0) * 1.5
    rng = np.random.default_rng(82)
    a = rng.normal(size=s.n_states)
    b = oracle.even_in_q(s, rng.normal(size=N0.shape))
    dt, n = 1.0, 3
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        f0, N0, a, b = (x.astype(np.float32).astype(np.float64) for x in (f0, N0, a, b))
        r, tdt, tol = round32(s), torch.float32, TOL32
    _, _, rf, rN, rg = oracle.rk4_coupled_trajectory_grad(r, f0, N0, dt, n, a, b)
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"coupled adjoint {name} {dtype} ce={ce}")
    gf, gN, gg = E.rt_adjoint_coupled(plan, dev(f0, tdt), dev(N0, tdt), dt, n, ce, dev(a, tdt), dev(b, tdt),
                                      gg2=True)
    plan.close()
    assert nerr(host(gf), rf) <= tol
    assert nerr(host(gN), rN) <= tol
    assert nerr(host(gg), rg) <= tol


def test_coupled_autograd(E):
    """CoupledSolve: the loss's gradients with respect to f0, N0 and |g|^2 from
    torch autograd equal the oracle's discrete adjoint; and the nph gradient of
    CollisionIntegral equals the oracle's."""
    from paper_2511_03683_amd.autograd import collision, coupled_solve
    s = synth.multiband_system()
    plan = E.build_channels(s, device=0)
    f0 = dev(0.1 + 0.8 * synth.random_occupations(s, 91)).requires_grad_(True)
    N0 = dev(s.nph(300.0) * 1.5).requires_grad_(True)
    g2 = dev(s.g2).requires_grad_(True)
    eps = dev(s.eps)
    say("coupled autograd")
    fT, NT = coupled_solve(f0, N0, g2, plan, 1.0, 3, 2)
    L = (eps * fT).sum() / fT.sum() + 0.01 * NT.sum()
    L.backward()
    fTh = host(fT)
    gT = (s.eps * fTh.sum() - s.eps @ fTh) / fTh.sum() ** 2
    gNT = np.full(s.hw.shape, 0.01)
    _, _, rf, rN, rg = oracle.rk4_coupled_trajectory_grad(s, host(f0), host(N0), 1.0, 3, gT, gNT)
    assert nerr(host(f0.grad), rf) <= TOL64
    assert nerr(host(N0.grad), rN) <= TOL64
    assert nerr(host(g2.grad), rg) <= TOL64
    f = dev(synth.random_occupations(s, 92))
    N = dev(_uneven_bath(s, 93)).requires_grad_(True)
    lam = np.random.default_rng(94).normal(size=s.n_states)
    (collision(f, dev(s.g2), plan, N) * dev(lam)).sum().backward()
    assert nerr(host(N.grad), oracle.collision_vjp_nph(s, host(f), host(N), lam)) <= TOL64
    plan.close()


def test_full_size_coupled_adjoint_finite_differences(E, c2):
    """dL/dN0 and dL/df0 through 5 coupled RK4 steps of 1 fs of the full-size
    system (L = mean carrier energy plus the mean phonon occupation at the
    end), against central differences along a random even direction of N0
    and a random direction of f0."""
    s = c2
    rng = np.random.default_rng(95)
    f0 = dev(synth.pulse_occupations(s, center=0.2))
    N0 = dev(s.nph(300.0))
    eps = dev(s.eps)
    dt, n = 1.0, 5
    plan = E.build_channels(s, device=0)

    def loss(ff, NN):
        ff, NN = ff.clone(), NN.clone()
        E.rt_step_coupled(plan, ff, NN, dt, n)
        torch.cuda.synchronize()
        return float((eps * ff).sum() / ff.sum() + NN.mean()), ff, NN

    say("full-size coupled adjoint vs finite differences")
    L0, fT, NT = loss(f0, N0)
    gT = ((eps * fT.sum() - (eps * fT).sum()) / fT.sum() ** 2).contiguous()
    gNT = torch.full_like(NT, 1.0 / NT.numel())
    gf, gN, _ = E.rt_adjoint_coupled(plan, f0, N0, dt, n, 2, gT, gNT)
    V = dev(oracle.even_in_q(s, rng.normal(size=s.hw.shape) * s.nph(300.0)))
    h = 1e-4
    fd = (loss(f0, N0 + h * V)[0] - loss(f0, N0 - h * V)[0]) / (2 * h)
    assert fd == pytest.approx(float((gN * V).sum()), rel=1e-5)
    v = dev(rng.normal(size=s.n_states) * 1e-2)
    fd = (loss(f0 + h * v, N0)[0] - loss(f0 - h * v, N0)[0]) / (2 * h)
    assert fd == pytest.approx(float((gf * v).sum()), rel=1e-5)
    plan.close()


def test_autograd_function(E):
    from paper_2511_03683_amd.autograd import collision
    s = synth.multiband_system()
    plan = E.build_channels(s, device=0)
    f = dev(synth.random_occupations(s, 1)).requires_grad_(True)
    g2 = dev(s.g2).requires_grad_(True)
    nph = dev(s.nph(300.0))
    lam = dev(np.random.default_rng(0).normal(size=s.n_states))
    say("autograd collision")
    L = (collision(f, g2, plan, nph) * lam).sum()
    L.backward()
    rf, rg = oracle.collision_vjp(s, host(f), s.nph(300.0), host(lam))
    assert nerr(host(f.grad), rf) <= TOL64
    assert nerr(host(g2.grad), rg) <= TOL64
    # an FP32 |g|^2 leaf receives its gradient in FP32
    g32 = dev(s.g2, torch.float32).requires_grad_(True)
    (collision(f.detach(), g32, plan, nph) * lam).sum().backward()
    assert g32.grad.dtype == torch.float32
    assert nerr(host(g32.grad), rg) <= 1e-6
    plan.close()


def test_update_g2(E):
    s = synth.multiband_system()
    f = synth.random_occupations(s, 3)
    nph = s.nph(300.0)
    plan = E.build_channels(s, device=0)
    g_new = s.g2 * np.linspace(0.5, 2.0, s.n_channels)
    say("update_g2")
    E.update_g2(plan, dev(g_new))
    I = host(E.collision_integral(plan, dev(f), dev(nph)))
    assert nerr(I, oracle.collision(s, f, nph, g2=g_new)) <= TOL64
    plan.close()


def test_kernel_timing(E):
    """The forward kernel's launch timing: one timed launch per eager call,
    none under graph capture, none once stopped."""
    s = synth.multiband_system()
    plan = E.build_channels(s, device=0)
    f, nph = dev(synth.random_occupations(s, 2)), dev(s.nph(300.0))
    say("kernel timing")
    E.kernel_timing(plan, True)
    for _ in range(3):
        E.collision_integral(plan, f, nph)
    ms, n = E.kernel_timing(plan, False)
    assert n == 3 and 0.0 < ms < 1000.0
    E.kernel_timing(plan, True)
    fe = dev(synth.random_occupations(s, 3))
    E.rt_step(plan, fe, nph, 0.5, 2, use_graph=False)   # 2 steps x 4 stages, eager
    E.rt_step(plan, fe, nph, 0.5, 4, use_graph=True)    # captured and replayed: not timed
    ms, n = E.kernel_timing(plan, False)
    assert n == 8 and ms > 0.0
    E.collision_integral(plan, f, nph)
    assert E.kernel_timing(plan, False) == (0.0, 0)
    plan.close()


# ------------------------------------------------------------------ RK4
def test_rt_step_matches_oracle_and_graph_replay(E):
    s = synth.multiband_system()
    nph = s.nph(300.0)
    f0 = synth.random_occupations(s, 7)
    dt, n = 0.5, 6
    ref = f0.copy()
    for _ in range(n):
        ref = oracle.rk4_step(s, ref, nph, dt)
    plan = E.build_channels(s, device=0)
    say("rt_step eager/graph")
    fe = dev(f0)
    E.rt_step(plan, fe, dev(nph), dt, n, use_graph=False)
    assert nerr(host(fe) - f0, ref - f0) <= TOL64
    fg = dev(f0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        E.rt_step(plan, fg, dev(nph), dt, n, use_graph=True)
        E.rt_step(plan, fg, dev(nph), dt, 0, use_graph=True)
    stream.synchronize()
    assert np.array_equal(host(fg), host(fe)), "graph replay is bitwise equal to eager"
    # replay the cached graph again and compare with eager twice as long
    fe2 = dev(f0)
    E.rt_step(plan, fe2, dev(nph), dt, 2 * n, use_graph=False)
    with torch.cuda.stream(stream):
        E.rt_step(plan, fg, dev(nph), dt, n, use_graph=True)
    stream.synchronize()
    assert np.array_equal(host(fg), host(fe2))
    # batch of two vectors, null stream graph path
    F = np.stack([f0, synth.random_occupations(s, 8)])
    Ft = dev(F)
    E.rt_step(plan, Ft, dev(nph), dt, n, use_graph=True)
    ref1 = F[1].copy()
    for _ in range(n):
        ref1 = oracle.rk4_step(s, ref1, nph, dt)
    got = host(Ft)
    # B = 2 runs the per-row pass, B = 1 the single-copy one: equal to rounding
    assert nerr(got[0] - f0, ref - f0) <= TOL64
    assert nerr(got[1] - F[1], ref1 - F[1]) <= TOL64
    plan.close()


def test_rt_adjoint_matches_oracle(E):
    s = synth.multiband_system(n_k=10, seed=23)
    f0 = synth.random_occupations(s, 9) * 0.8 + 0.1
    nph = s.nph(300.0)
    dt, n = 0.5, 5
    gT = np.random.default_rng(5).normal(size=s.n_states)
    _, rf, rg = oracle.rk4_trajectory_grad(s, f0, nph, dt, n, gT)
    plan = E.build_channels(s, device=0)
    say("rt_adjoint")
    outs = []
    for ce in (1, 2, 5):
        gf0, gg = E.rt_adjoint(plan, dev(f0), dev(nph), dt, n, ce, dev(gT), gg2=True)
        outs.append((host(gf0), host(gg)))
        assert nerr(outs[-1][0], rf) <= TOL64
        assert nerr(outs[-1][1], rg) <= TOL64
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1]), \
            "checkpointing does not change the gradient"
    plan.close()


RATES = np.array([0.06, -0.035, 0.02])   # 1/fs: a strong field, so the drift is felt in a few steps


@pytest.mark.parametrize("dtype,B", [("f64", 1), ("f64", 3), ("f64", 9), ("f32", 1)])
def test_rt_step_with_field(E, dtype, B):
    """Eq. 1 with the field term: RK4 with collisions and drift against the
    oracle (single-copy, per-row and batched forward passes, eager and graph);
    a zero field gives back the field-free step bitwise."""
    s = synth.multiband_system()
    nph = s.nph(300.0)
    F = np.stack([synth.random_occupations(s, 30 + b) for b in range(B)])
    dt, n = 1.0, 4
    r, tdt, tol = s, torch.float64, TOL64
    if dtype == "f32":
        F, nph = F.astype(np.float32).astype(np.float64), nph.astype(np.float32).astype(np.float64)
        r, tdt, tol = round32(s), torch.float32, 1e-5
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"rt_step field {dtype} B={B}")
    E.set_field(plan, RATES)
    ft = dev(F if B > 1 else F[0], tdt)
    E.rt_step(plan, ft, dev(nph, tdt), dt, n, use_graph=False)
    got = host(ft).reshape(B, -1)
    for b in range(B):
        ref = F[b].copy()
        for _ in range(n):
            ref = oracle.rk4_step(r, ref, nph, dt, rates=RATES)
        assert nerr(got[b] - F[b], ref - F[b]) <= tol, b
    fg = dev(F if B > 1 else F[0], tdt)
    E.rt_step(plan, fg, dev(nph, tdt), dt, n, use_graph=True)
    assert np.array_equal(host(fg), host(ft))
    E.set_field(plan, [0.0, 0.0, 0.0])
    f1, f2 = dev(F[0], tdt), dev(F[0], tdt)
    E.rt_step(plan, f1, dev(nph, tdt), dt, n)
    plan2 = E.build_channels(s, dtype=dtype, device=0)
    E.rt_step(plan2, f2, dev(nph, tdt), dt, n)
    assert np.array_equal(host(f1), host(f2))
    plan.close()
    plan2.close()


def test_rt_adjoint_with_field(E):
    """Discrete adjoint through RK4 steps with collisions and drift against the
    oracle's (whose drift transpose is the scattered matrix, not -D)."""
    s = synth.multiband_system(n_k=10, seed=23)
    f0 = synth.random_occupations(s, 9) * 0.8 + 0.1
    nph = s.nph(300.0)
    dt, n = 1.0, 4
    gT = np.random.default_rng(6).normal(size=s.n_states)
    _, rf, rg = oracle.rk4_trajectory_grad(s, f0, nph, dt, n, gT, rates=RATES)
    plan = E.build_channels(s, device=0)
    E.set_field(plan, RATES)
    say("rt_adjoint field")
    gf0, gg = E.rt_adjoint(plan, dev(f0), dev(nph), dt, n, 2, dev(gT), gg2=True)
    assert nerr(host(gf0), rf) <= TOL64
    assert nerr(host(gg), rg) <= TOL64
    plan.close()


def test_field_term_arguments(E):
    """set_field refuses non-finite rates, and nonzero rates on a plan where a
    (k, band) is held by two states; zero rates give back the field-free step."""
    import copy
    s = synth.multiband_system()
    plan = E.build_channels(s, device=0)
    say("field term arguments")
    with pytest.raises(E.EphbteError, match="finite"):
        E.set_field(plan, [np.nan, 0.0, 0.0])
    nph = dev(s.nph(300.0))
    f1, f2 = dev(synth.random_occupations(s, 5)), dev(synth.random_occupations(s, 5))
    E.set_field(plan, RATES)
    E.set_field(plan, [0.0, 0.0, 0.0])
    E.rt_step(plan, f1, nph, 0.5, 2)
    plan2 = E.build_channels(s, device=0)
    E.rt_step(plan2, f2, nph, 0.5, 2)
    assert np.array_equal(host(f1), host(f2))
    plan.close()
    plan2.close()
    # without bands the two states of each k point share (k, band 0)
    nb = copy.copy(s)
    nb.state_band = np.zeros_like(s.state_band)
    plan = E.build_channels(nb, device=0)
    E.set_field(plan, [0.0, 0.0, 0.0])
    with pytest.raises(E.EphbteError, match="band"):
        E.set_field(plan, RATES)
    plan.close()


def test_rt_solve_autograd(E):
    from paper_2511_03683_amd.autograd import rt_solve
    s = synth.multiband_system(n_k=10, seed=23)
    plan = E.build_channels(s, device=0)
    f0 = dev(synth.random_occupations(s, 9) * 0.8 + 0.1).requires_grad_(True)
    g2 = dev(s.g2).requires_grad_(True)
    nph = dev(s.nph(300.0))
    eps = dev(s.eps)
    say("rt_solve autograd")
    fT = rt_solve(f0, g2, plan, nph, 0.5, 4, checkpoint_every=2)
    L = (eps * fT).sum() / fT.sum()
    L.backward()
    gT = host((eps * fT.sum() - (eps * fT).sum()) / fT.sum() ** 2)
    _, rf, rg = oracle.rk4_trajectory_grad(s, host(f0), s.nph(300.0), 0.5, 4, gT)
    assert nerr(host(f0.grad), rf) <= TOL64
    assert nerr(host(g2.grad), rg) <= TOL64
    plan.close()


# ------------------------------------------------------------------ transport
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_transport_matches_oracle(E, dtype):
    s = synth.tb_system(kn=20, qn=10, target_states=300, sigma=0.05)
    T = 300.0
    f0 = synth.fermi_dirac(s.eps, -0.1, T)
    nph = s.nph(T)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = E.build_channels(s, dtype=dtype, device=0)
    say(f"transport {dtype}")
    k = 7
    out = E.iterate_transport(plan, dev(f0, tdt), dev(s.vel, tdt), T, dev(nph, tdt), tol=0.0,
                              max_iter=k, want_x=True)
    assert not out["converged"] and out["iters"] == k
    if dtype == "f64":
        ref = oracle.transport_solve(s, f0, s.vel, T, nph, max_iter=k, stop_on_tol=False)
        assert nerr(out["mu"], ref["mu"]) <= TOL64
        assert nerr(host(out["x"]), ref["x"]) <= TOL64
        conv = E.iterate_transport(plan, dev(f0), dev(s.vel), T, dev(nph), tol=1e-10, max_iter=500)
        refc = oracle.transport_solve(s, f0, s.vel, T, nph, tol=1e-10, max_iter=500)
        assert conv["converged"] and conv["iters"] == refc["iters"]
        assert nerr(conv["mu"], refc["mu"]) <= TOL64
    else:
        r = round32(s)
        f32 = f0.astype(np.float32).astype(np.float64)
        ref = oracle.transport_solve(r, f32, s.vel.astype(np.float32).astype(np.float64), T,
                                     nph.astype(np.float32).astype(np.float64), max_iter=k,
                                     stop_on_tol=False)
        assert nerr(out["mu"], ref["mu"]) <= TOL32
        assert nerr(host(out["x"]), ref["x"]) <= TOL32
    plan.close()


def test_transport_fp32_stops_at_its_floor(E):
    """FP32 cannot resolve a 1e-12 change: the iteration stops on stagnation
    (reported as such) well before max_iter, with the mobility of the FP64
    fixed point to FP32 accuracy."""
    s = synth.tb_system(kn=20, qn=10, target_states=300, sigma=0.05)
    T = 300.0
    f0 = synth.fermi_dirac(s.eps, -0.1, T)
    nph = s.nph(T)
    plan = E.build_channels(s, dtype="f32", device=0)
    say("transport f32 stagnation stop")
    out = E.iterate_transport(plan, dev(f0, torch.float32), dev(s.vel, torch.float32), T,
                              dev(nph, torch.float32), tol=1e-12, max_iter=2000)
    # either the change stopped decreasing, or FP32 landed on an exact fixed point
    assert out["iters"] < 2000
    assert out["stagnated"] or (out["converged"] and out["resid"] == 0.0)
    ref = oracle.transport_solve(s, f0, s.vel, T, nph, tol=1e-12, max_iter=2000)
    assert ref["converged"]
    assert nerr(out["mu"], ref["mu"]) <= TOL32
    plan.close()


# ------------------------------------------------------------------ full size
# ---------------------------------------------------------------------------
# phonon-phonon scattering: Bose plans (statistics "bose")
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def phph():
    s = synth.ph_ph_system(n=6)
    n = synth.bose_occupations(s, 300.0, seed=80)
    return s, n, synth.bose_einstein(s.hw, 250.0)


def _bose_ref(s, n, nph, dtype):
    if dtype == "f64":
        return oracle.collision_bose(s, n, nph), TOL64, torch.float64, n, nph
    r = round32(s)
    n32, N32 = n.astype(np.float32).astype(np.float64), nph.astype(np.float32).astype(np.float64)
    return oracle.collision_bose(r, n32, N32), TOL32, torch.float32, n32, N32


@pytest.mark.parametrize("dtype,layout", [("f64", 3), ("f64", 2), ("f64", 1), ("f32", 3), ("f32", 1)])
def test_bose_forward_matches_oracle(E, phph, dtype, layout):
    """Three-phonon collision integral of a Bose plan (646 modes, 6.2e5
    channels) against the oracle's Bose integral, over each layout."""
    s, n, nph = phph
    ref, tol, tdt, n_in, N_in = _bose_ref(s, n, nph, dtype)
    plan = E.build_channels(s, dtype=dtype, device=0, statistics="bose")
    E.set_tuning(plan, layout=layout)
    say(f"bose forward {dtype} layout {layout} S={s.n_states} Nch={s.n_channels}")
    I = host(E.collision_integral(plan, dev(n_in, tdt), dev(N_in, tdt)))
    assert nerr(I, ref) <= tol
    plan.close()


def test_bose_forward_larger_grid(E):
    """An 8^3 grid (1534 modes, 3.5e6 channels), FP64 over pair records."""
    s = synth.ph_ph_system(n=8)
    n = synth.bose_occupations(s, 300.0, seed=81)
    nph = synth.bose_einstein(s.hw, 320.0)
    plan = E.build_channels(s, device=0, statistics="bose")
    say(f"bose forward 8^3 S={s.n_states} Nch={s.n_channels}")
    I = host(E.collision_integral(plan, dev(n), dev(nph)))
    assert nerr(I, oracle.collision_bose(s, n, nph)) <= TOL64
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bose_batched_reverse_and_baths(E, phph, dtype):
    """Bose plan, B = 9: forward and reverse (dL/dn per vector, dL/d|V|^2
    summed) through the batched kernels; B = 4 with a bath per vector; the
    reverse at B = 1 and dL/dN."""
    s, n0, nph = phph
    B = 9
    F = np.stack([synth.bose_occupations(s, 300.0, seed=90 + b) for b in range(B)])
    L = np.random.default_rng(91).normal(size=(B, s.n_states))
    r, tol, tdt = s, TOL64, torch.float64
    NPH = np.stack([synth.bose_einstein(s.hw, 200.0 + 50.0 * b) for b in range(4)])
    N1 = nph
    if dtype == "f32":
        F, L, NPH, N1 = (a.astype(np.float32).astype(np.float64) for a in (F, L, NPH, nph))
        r, tol, tdt = round32(s), TOL32, torch.float32
    plan = E.build_channels(s, dtype=dtype, device=0, statistics="bose")
    say(f"bose batched {dtype} B={B}")
    I = host(E.collision_integral(plan, dev(F, tdt), dev(N1, tdt)))
    for b in range(B):
        assert nerr(I[b], oracle.collision_bose(r, F[b], N1)) <= tol, b
    gf, gg = E.collision_vjp(plan, dev(F, tdt), dev(N1, tdt), dev(L, tdt), gg2=True)
    gf, gg = host(gf), host(gg)
    rg = 0
    for b in range(B):
        rn, rg_b, _ = oracle.collision_bose_vjp(r, F[b], N1, L[b])
        assert nerr(gf[b], rn) <= tol, b
        rg = rg + rg_b
    assert nerr(gg, rg) <= tol
    say(f"bose bath per vector {dtype}")
    I4 = host(E.collision_integral(plan, dev(F[:4], tdt), dev(NPH, tdt)))
    for b in range(4):
        assert nerr(I4[b], oracle.collision_bose(r, F[b], NPH[b])) <= tol, b
    say(f"bose reverse B=1 and dL/dN {dtype}")
    gf1, gg1 = E.collision_vjp(plan, dev(F[0], tdt), dev(N1, tdt), dev(L[0], tdt), gg2=True)
    rn, rg1, rN = oracle.collision_bose_vjp(r, F[0], N1, L[0])
    assert nerr(host(gf1), rn) <= tol
    assert nerr(host(gg1), rg1) <= tol
    gN = host(E.collision_vjp_nph(plan, dev(F[0], tdt), dev(N1, tdt), dev(L[0], tdt)))
    assert nerr(gN, rN) <= tol
    plan.close()


def test_bose_rt_steps_and_adjoint(E, phph):
    """RK4 steps of dn/dt = I_B[n] (eager and graph replay, bitwise equal)
    and their checkpointed adjoint, against the oracle."""
    s, n0, nph = phph
    dt, steps = 200.0, 4
    ref = n0.copy()
    for _ in range(steps):
        ref = oracle.rk4_step(s, ref, nph, dt, statistics="bose")
    plan = E.build_channels(s, device=0, statistics="bose")
    say("bose rt steps")
    a, b = dev(n0), dev(n0)
    E.rt_step(plan, a, dev(nph), dt, steps)
    E.rt_step(plan, b, dev(nph), dt, steps, use_graph=True)
    a, b = host(a), host(b)
    assert np.array_equal(a, b)
    assert nerr(a - n0, ref - n0) <= TOL64
    gT = np.random.default_rng(92).normal(size=s.n_states)
    _, rn, rg = oracle.rk4_trajectory_grad(s, n0, nph, dt, 3, gT, statistics="bose")
    say("bose rt adjoint")
    for ce in (1, 3):
        gn, gg = E.rt_adjoint(plan, dev(n0), dev(nph), dt, 3, ce, dev(gT), gg2=True)
        assert nerr(host(gn), rn) <= TOL64
        assert nerr(host(gg), rg) <= TOL64
    plan.close()


def test_bose_plan_rejects_fermi_only_entry_points(E, phph):
    s, n0, nph = phph
    plan = E.build_channels(s, device=0, statistics="bose")
    say("bose rejections")
    with pytest.raises(E.EphbteError, match="Fermi statistics only"):
        E.phonon_rate(plan, dev(n0), dev(nph))
    with pytest.raises(E.EphbteError, match="Fermi statistics only"):
        E.set_field(plan, [0.01, 0.0, 0.0])
    with pytest.raises(E.EphbteError, match="Fermi statistics only"):
        E.collision_integral_noalloc(plan, dev(n0), dev(nph), dev(np.zeros(s.n_states)))
    with pytest.raises(ValueError):
        E.build_channels(s, device=0, statistics="anyon")
    plan.close()


@pytest.fixture(scope="module")
def c2():
    return synth.tb_system()


def full_norm(r, f, nph, ref, dtype, args=None):
    """Norm of the full-vector error: max|I_ref| (FP64); for FP32
    max(max|I_ref|, 1e-2 max(in, out)) over every state, from the oracle
    (reading 15: a near-equilibrium vector is judged against its gross rates)."""
    if dtype == "f64":
        return np.abs(ref).max()
    rin, rout = oracle.collision_inout_threads(r, f, nph, args=args)
    return max(np.abs(ref).max(), 1e-2 * max(rin.max(), rout.max()))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_parity(E, c2, dtype):
    """The 100^3/50^3, ~2e8-channel system in the launch configuration the
    benchmark times, every output against the oracle's channel loop over the
    whole list (run on all host threads)."""
    s = c2
    rng = np.random.default_rng(17)
    f = np.clip(synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
    say(f"full-size {dtype} S={s.n_states} Nch={s.n_channels}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    plan.close()
    r = s if dtype == "f64" else round32(s)
    a = oracle._Args(r, nph)
    ref = oracle.collision_threads(r, f, nph, args=a)
    say(f"full-size {dtype} oracle done")
    assert np.isfinite(I).all()
    if dtype == "f64":
        assert abs(I.sum()) <= 1e-10 * np.abs(I).sum()
    assert nerr(I, ref, full_norm(r, f, nph, ref, dtype, args=a)) <= (TOL64 if dtype == "f64" else TOL32)


@pytest.fixture(scope="module")
def c2b():
    return synth.tb_two_band_system()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_two_band_parity(E, c2b, dtype):
    """The two-band variant of the full-size workload (two bands in the 0.3 eV
    window, inter-band channels, pair records with partly filled mode slots):
    every output of the default B = 1 pass against the oracle's channel loop
    over the whole list."""
    s = c2b
    rng = np.random.default_rng(19)
    assert len(np.unique(s.state_band)) == 2
    f = np.clip(synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    r = s
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
        r = round32(s)
    say(f"full-size two-band {dtype} S={s.n_states} Nch={s.n_channels}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    plan.close()
    a = oracle._Args(r, nph)
    ref = oracle.collision_threads(r, f, nph, args=a)
    assert np.isfinite(I).all()
    assert nerr(I, ref, full_norm(r, f, nph, ref, dtype, args=a)) <= (TOL64 if dtype == "f64" else TOL32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_batched_parity(E, c2, dtype):
    """B = 64 vectors of the full-size system in one pass, as the benchmark
    times it; two columns checked in full against the oracle's channel loop
    over the whole list; every column within the per-state bound."""
    s = c2
    rng = np.random.default_rng(23)
    B = 64
    base = synth.fermi_dirac(s.eps, 0.05, 300.0)
    F = np.clip(base[None, :] * rng.uniform(0.7, 1.3, size=(B, 1)), 0, 1)
    F[7] = np.clip(base * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        F = F.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
    say(f"full-size batched {dtype} B={B}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    I = host(E.collision_integral(plan, dev(F, tdt), dev(nph, tdt)))
    plan.close()
    plausible(I, rate_bound(s, nph)[None, :])
    r = s if dtype == "f64" else round32(s)
    a = oracle._Args(r, nph)
    for b in (7, 63):
        ref = oracle.collision_threads(r, F[b], nph, args=a)
        err = nerr(I[b], ref, full_norm(r, F[b], nph, ref, dtype, args=a))
        assert err <= (TOL64 if dtype == "f64" else TOL32), b


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_batched_vjp_sampled_parity(E, c2, dtype):
    """The B = 64 reverse pass on the full-size system, as the benchmark times
    it.  dL/df_d needs only the channels touching d and each dL/d|g|^2 only
    its own channel, so the oracle runs on the channels incident to 24
    sampled destinations, for all 64 vectors."""
    s = c2
    rng = np.random.default_rng(29)
    B = 64
    F = synth.batch_occupations(s)
    L = rng.normal(size=(B, s.n_states))
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        F, L, nph = (a.astype(np.float32).astype(np.float64) for a in (F, L, nph))
    say(f"full-size batched reverse {dtype} B={B}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    gf, gg = E.collision_vjp(plan, dev(F, tdt), dev(nph, tdt), dev(L, tdt), gg2=True)
    gf, gg = host(gf), host(gg)
    plan.close()
    dests = rng.choice(s.n_states, 24, replace=False)
    inc = np.isin(s.ch_i, dests) | np.isin(s.ch_j, dests)
    sub = oracle.subset(s if dtype == "f64" else round32(s), inc)
    rf = np.zeros((B, s.n_states))
    rg = np.zeros(int(inc.sum()))
    for b in range(B):
        f_b, g_b = oracle.collision_vjp(sub, F[b], nph, L[b])
        rf[b] = f_b
        rg += g_b
    tol = TOL64 if dtype == "f64" else TOL32
    assert np.isfinite(gf).all() and np.isfinite(gg).all()
    assert nerr(gf[:, dests], rf[:, dests]) <= tol
    assert nerr(gg[inc], rg) <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_vjp_sampled_parity(E, c2, dtype):
    """The B = 1 reverse pass on the full-size system: dL/df on 32 sampled
    destinations and dL/d|g|^2 of every channel touching them, from the oracle
    on those incident channels."""
    s = c2
    rng = np.random.default_rng(37)
    f = np.clip(synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    lam = rng.normal(size=s.n_states)
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        f, lam, nph = (a.astype(np.float32).astype(np.float64) for a in (f, lam, nph))
    say(f"full-size reverse {dtype}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    gf, gg = E.collision_vjp(plan, dev(f, tdt), dev(nph, tdt), dev(lam, tdt), gg2=True)
    gf, gg = host(gf), host(gg)
    plan.close()
    dests = rng.choice(s.n_states, 32, replace=False)
    inc = np.isin(s.ch_i, dests) | np.isin(s.ch_j, dests)
    rf, rg = oracle.collision_vjp(oracle.subset(s if dtype == "f64" else round32(s), inc), f, nph, lam)
    tol = TOL64 if dtype == "f64" else TOL32
    assert np.isfinite(gf).all() and np.isfinite(gg).all()
    assert nerr(gf[dests], rf[dests]) <= tol
    assert nerr(gg[inc], rg) <= tol


def test_full_size_phonon_rate_sampled_parity(E, c2):
    """dN/dt of the full-size system (FP64): a bin depends only on the
    channels whose q or -q falls in it, so the oracle runs on the channels of
    12 sampled (q, mode) bins and their partners at -q."""
    s = c2
    rng = np.random.default_rng(41)
    f = np.clip(synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    nph = s.nph(300.0)
    say("full-size phonon rate")
    plan = E.build_channels(s, device=0)
    dN = host(E.phonon_rate(plan, dev(f), dev(nph)))
    plan.close()
    kg = np.asarray(s.kgrid, np.int64)
    qg = np.asarray(s.qgrid, np.int64)
    kc = synth.grid_coords(s.kgrid)[s.state_k].astype(np.int32)
    r = (kg // qg).astype(np.int32)
    qlin = np.zeros(s.n_channels, np.int64)
    for a in range(3):
        qa = ((kc[s.ch_j, a] - kc[s.ch_i, a]) % int(kg[a])) // int(r[a])
        qlin = qlin * int(qg[a]) + qa
    qneg = np.zeros(s.n_channels, np.int64)
    for a in range(3):
        qa = ((kc[s.ch_i, a] - kc[s.ch_j, a]) % int(kg[a])) // int(r[a])
        qneg = qneg * int(qg[a]) + qa
    nm = s.n_modes
    pick = rng.choice(s.n_channels, 12, replace=False)
    bins = np.unique(np.concatenate([qlin[pick] * nm + s.ch_nu[pick], qneg[pick] * nm + s.ch_nu[pick]]))
    keep = np.isin(qlin * nm + s.ch_nu, bins) | np.isin(qneg * nm + s.ch_nu, bins)
    ref = oracle.phonon_rate(oracle.subset(s, keep), f, nph).reshape(-1)
    got = dN.reshape(-1)
    assert np.abs(ref[bins]).max() > 0
    assert np.isfinite(got).all()
    assert nerr(got[bins], ref[bins]) <= TOL64


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_transport_iteration(E, c2, dtype):
    """One transport iteration of the full-size system in the launch
    configuration the benchmark times: x after k + 1 iterations at 32 sampled
    destinations against the oracle's update x_d = tau_d (v_d df0/de +
    sum_p W_dp x_p) of the GPU's x after k iterations (tau and W of a
    destination need only its incident channels), and the mobility against
    the host sum over the GPU's x."""
    s = c2
    T = 300.0
    f0 = synth.fermi_dirac(s.eps, -0.1, T)
    nph = s.nph(T)
    vel = np.asarray(s.vel, np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    r = s
    if dtype == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
        vel = vel.astype(np.float32).astype(np.float64)
        r = round32(s)
    say(f"full-size transport iteration {dtype}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    k = 3
    outs = [E.iterate_transport(plan, dev(f0, tdt), dev(vel, tdt), T, dev(nph, tdt), tol=0.0,
                                max_iter=n, want_x=True) for n in (k, k + 1)]
    plan.close()
    xk, xk1 = host(outs[0]["x"]), host(outs[1]["x"])
    rng = np.random.default_rng(53)
    dests = rng.choice(s.n_states, 32, replace=False)
    sub = oracle.subset(r, incident(s, dests))
    tau_inv, Wij, Wji = oracle.transport_coeffs(sub, f0, nph)
    b = vel * oracle.dfde_fd(f0, T)[:, None]
    ref = (b + oracle.transport_apply_W(sub, Wij, Wji, xk))[dests] / tau_inv[dests, None]
    tol = TOL64 if dtype == "f64" else TOL32
    assert np.isfinite(xk1).all()
    assert nerr(xk1[dests], ref) <= tol
    assert nerr(outs[1]["mu"], oracle.mobility_cm2(vel, xk1, f0)) <= tol


# ------------------------------------------------------------------ uneven batch
@pytest.fixture(scope="module")
def grouped():
    return synth.grouped_system()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_grouped_uneven_systems_one_launch(E, grouped, dtype):
    """16 systems of 1e5 .. 1e7 channels concatenated into one problem and
    evaluated by one launch; every system's output against the oracle's
    channel loop, each normalised by its own vector (normwise per system)."""
    s = grouped
    rng = np.random.default_rng(31)
    f = np.clip(synth.fermi_dirac(s.eps, 0.05, 300.0) * (0.8 + 0.4 * rng.uniform(size=s.n_states)), 0, 1)
    nph = s.nph(300.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
        nph = nph.astype(np.float32).astype(np.float64)
    say(f"grouped {dtype} S={s.n_states} Nch={s.n_channels}")
    plan = E.build_channels(s, dtype=dtype, device=0)
    I = host(E.collision_integral(plan, dev(f, tdt), dev(nph, tdt)))
    plan.close()
    offs = s.meta["offsets"]
    r = s if dtype == "f64" else round32(s)
    a = oracle._Args(r, nph)
    ref = oracle.collision_threads(r, f, nph, args=a)
    if dtype == "f32":
        rin, rout = oracle.collision_inout_threads(r, f, nph, args=a)
    assert np.isfinite(I).all()
    for m in range(len(offs) - 1):
        sl = slice(offs[m], offs[m + 1])
        if dtype == "f64":
            assert nerr(I[sl], ref[sl]) <= TOL64, m
        else:
            scale = max(np.abs(ref[sl]).max(), 1e-2 * max(rin[sl].max(), rout[sl].max()))
            assert nerr(I[sl], ref[sl], scale) <= TOL32, m


# ------------------------------------------------------------------ gradients
def test_rt_adjoint_cpu_reference_512k(E):
    """Gradient through 6 RK4 steps on the 512-k case against the oracle's
    discrete adjoint (FP64)."""
    s = synth.parabolic_system(8)
    f0 = synth.c1_occupations(s)
    nph = s.nph(300.0)
    dt, n = 1.0, 6
    fT = f0.copy()
    for _ in range(n):
        fT = oracle.rk4_step(s, fT, nph, dt)
    gT = (s.eps * fT.sum() - s.eps @ fT) / fT.sum() ** 2
    _, rf, rg = oracle.rk4_trajectory_grad(s, f0, nph, dt, n, gT)
    plan = E.build_channels(s, device=0)
    say("rt_adjoint 512-k vs oracle")
    gf0, gg = E.rt_adjoint(plan, dev(f0), dev(nph), dt, n, 2, dev(gT), gg2=True)
    plan.close()
    assert nerr(host(gf0), rf) <= TOL64
    assert nerr(host(gg), rg) <= TOL64


def test_full_size_rt_adjoint_finite_differences(E, c2):
    """dL/d|g|^2 through 200 RK4 steps of 1 fs (checkpoint every 20) of the
    full-size system, the pulse inside the energy window, L = mean carrier
    energy at 200 fs, against central differences on the 32 entries of
    largest |dL/dg2| and along one random direction."""
    s = c2
    nph = dev(s.nph(300.0))
    eps = dev(s.eps)
    f0 = dev(synth.pulse_occupations(s, center=0.2))
    dt, n = 1.0, 200
    plan = E.build_channels(s, device=0)
    g2 = dev(s.g2)

    def loss(g):
        E.update_g2(plan, g)
        f = f0.clone()
        E.rt_step(plan, f, nph, dt, n, use_graph=True)
        torch.cuda.synchronize()
        return float((eps * f).sum() / f.sum()), f

    say("full-size adjoint vs finite differences")
    L0, fT = loss(g2)
    gT = ((eps * fT.sum() - (eps * fT).sum()) / fT.sum() ** 2).contiguous()
    _, gg = E.rt_adjoint(plan, f0, nph, dt, n, 20, gT, want_f=False, gg2=True)
    gg = host(gg)
    top = np.argsort(-np.abs(gg))[:32]
    for k, c in enumerate(top):
        if k % 8 == 0:
            say(f"finite differences {k} / 32")
        h = 1e-2 * s.g2[c]
        gp = g2.clone()
        gp[c] += h
        gm = g2.clone()
        gm[c] -= h
        fd = (loss(gp)[0] - loss(gm)[0]) / (2 * h)
        assert fd == pytest.approx(gg[c], rel=2e-3, abs=1e-3 * np.abs(gg[top]).max()), c
    v = np.random.default_rng(3).normal(size=s.n_channels) * s.g2
    hstep = 1e-3
    Lp = loss(g2 + hstep * dev(v))[0]
    Lm = loss(g2 - hstep * dev(v))[0]
    fd = (Lp - Lm) / (2 * hstep)
    assert fd == pytest.approx(float(gg @ v), rel=1e-4)
    plan.close()
