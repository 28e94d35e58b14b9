"""The allocation-free forward pass (ephbte_collision_integral_noalloc),
called through the C ABI, against the plain entry point
(ephbte_collision_integral) and the FP64 oracle: two calls in a row on one
GPU, the second on a smaller system, so the second call reuses the static
scratch the first one filled."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-5


def say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _tensor(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _both(E, s, f, nph, dtype):
    """(plain, allocation-free) results of one plan through the C ABI."""
    lib = E.load_library()
    dt = torch.float64 if dtype == "f64" else torch.float32
    plan = E.build_channels(s, dtype=dtype, device=0)
    ft, nt = _tensor(f, dt), _tensor(nph, dt)
    I = torch.full((s.n_states,), float("nan"), dtype=dt, device="cuda:0")
    J = torch.full((s.n_states,), float("nan"), dtype=dt, device="cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.ephbte_collision_integral(plan.handle, 1, ft.data_ptr(), s.n_states, nt.data_ptr(), 0,
                                       I.data_ptr(), s.n_states, stream)
    assert st == 0, E.last_error()
    st = lib.ephbte_collision_integral_noalloc(plan.handle, ft.data_ptr(), nt.data_ptr(), J.data_ptr(),
                                               stream)
    assert st == 0, E.last_error()
    out = _host(I), _host(J)
    plan.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_allocation_free_pass_matches_plain_pass(dtype):
    import paper_2511_03683_amd as E
    assert torch.cuda.is_available()
    big = synth.tb_system(kn=24, qn=12, target_states=400)
    small = synth.multiband_system()
    tol = TOL64 if dtype == "f64" else TOL32
    for s, seed in ((big, 6), (small, 4)):
        say(f"noalloc {dtype} {s.name} S={s.n_states} channels={s.n_channels}")
        f = 0.05 + 0.9 * synth.random_occupations(s, seed)
        nph = s.nph(300.0)
        I, J = _both(E, s, f, nph, dtype)
        assert np.isfinite(J).all()
        err = np.abs(J - I).max() / np.abs(I).max()
        print(f"[gpu-err] noalloc vs plain {err:.3e}", flush=True)
        assert err <= tol
        if dtype == "f64":
            ref = oracle.collision(s, f, nph)
            assert np.abs(J - ref).max() / np.abs(ref).max() <= TOL64
