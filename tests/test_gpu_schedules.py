"""The paired stencil schedule (S1+S2 and S3+S4 each in one pass, LDS-staged
planes with a one-cell halo recompute) against the oracle and against the
five-pass schedule, through the C ABI, on ragged shapes and every tile."""
import numpy as np
import pytest

import oracle
import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402
from test_gpu_parity import T_STAR, rand_problem, rel  # noqa: E402


def run(p, mask, phi, T, dt, steps, precision, schedule, tile=None, use_graph=True):
    s = pf.Solver(p, mask, precision, dict(tol=0.0))
    s.set_schedule(schedule)
    s.set_loop(5, use_graph)
    npdt = np.float64 if precision == "fp64" else np.float32
    s.set_state(phi.astype(npdt), None if p["model"] == "ac" else (T - T_STAR).astype(npdt))
    s.set_time(0.0, dt)
    st = s.integrate(max_steps=steps)
    out = s.get_state() + (st, s.diagnostics(), s.get_config())
    s.close()
    return out


SHAPES = [(19, 13, 70), (9, 17, 33), (40, 5, 3), (6, 1, 1), (1, 1, 7), (33, 66, 129)]


@pytest.mark.parametrize("model,dt", [("ac", 0.5), ("coupled", 2e-3)])
@pytest.mark.parametrize("shape", SHAPES)
def test_paired_fp64_matches_oracle(model, dt, shape):
    p, mask, phi, T = rand_problem(shape, model, 31, faces=(1 << 4) | 1, bc_kind=1)
    steps = 6
    P = oracle.make_params(p)
    ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt, phi,
                                    T if model == "coupled" else None, max_steps=steps)
    ph, th, st, d, cfg = run(p, mask, phi, T, dt, steps, "fp64", "paired")
    assert cfg["schedule"] == "paired" and cfg["passes"] == 3
    assert st["steps_accepted"] == steps
    assert rel(ph, ph_o) <= 1e-12
    if model == "coupled":
        assert rel(th, T_o - T_STAR) <= 1e-12
    od = oracle.diagnostics(P, mask, ph_o, T_o)
    assert d["ice_count"] == od["ice_count"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("model", ["ac", "coupled"])
def test_paired_equals_five_pass(precision, model):
    p, mask, phi, T = rand_problem((37, 22, 75), model, 9, faces=1 << 4, bc_kind=1)
    dt = 2e-3 if model == "coupled" else 0.5
    a = run(p, mask, phi, T, dt, 12, precision, "paired")
    b = run(p, mask, phi, T, dt, 12, precision, "five")
    tol = 1e-13 if precision == "fp64" else 2e-6
    assert rel(a[0], b[0]) <= tol
    if model == "coupled":
        assert rel(a[1], b[1]) <= tol
    assert a[2]["sum_phi"] == pytest.approx(b[2]["sum_phi"], rel=1e-12 if precision == "fp64" else 1e-6)


def test_paired_adaptive_diagnostics_match_five_pass():
    c = pi.crop_case(pi.case_coupled_128(), lo=(30, 40, 0), size=(70, 50, 40))
    outs = []
    for sched in ("paired", "five"):
        s = pf.Solver(c.params, c.mask, "fp64", c.run)
        s.set_schedule(sched)
        s.set_state(c.phi0, c.T0 - T_STAR)
        s.set_time(0.0, 1e-4)
        st = s.integrate(max_steps=120)
        outs.append((s.get_state(), st))
        s.close()
    (pa, sa), (pb, sb) = outs
    assert sa["steps_accepted"] == sb["steps_accepted"]
    assert sa["steps_rejected"] == sb["steps_rejected"]
    # roundoff-sized error estimates of the first attempts make the step
    # sequences drift apart at the 1e-12 level per step (as oracle vs GPU)
    gaps = (rel(pa[0], pb[0]), rel(pa[1], pb[1]))
    assert max(gaps) <= 1e-8, gaps
    assert sa["ice_count"] == sb["ice_count"]


@pytest.mark.parametrize("ts", [0, 1, 2])
@pytest.mark.parametrize("zc", [4, 7, 64])
def test_every_pair_tile_matches_oracle(ts, zc):
    p, mask, phi, T = rand_problem((23, 41, 67), "coupled", 50 + ts, faces=(1 << 4) | (1 << 2))
    P = oracle.make_params(p)
    ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, 2e-3, phi, T,
                                    max_steps=4)
    s = pf.Solver(p, mask, "fp64", dict(tol=0.0))
    s.set_schedule("paired")
    s.set_pair_tile(ts, zc)
    s.set_state(phi, T - T_STAR)
    s.set_time(0.0, 2e-3)
    s.integrate(max_steps=4)
    ph, th = s.get_state()
    cfg = s.get_config()
    s.close()
    assert cfg["pair_z_chunk"] == min(max(zc, 4), 23)
    assert rel(ph, ph_o) <= 1e-12 and rel(th, T_o - T_STAR) <= 1e-12


# n1 = 260 (65 FP32 / 130 FP64 vectors per row: rows straddle wavefronts);
# n1 = 6 and 130: FP64 vectors only (n1 not divisible by 4)
VEC_SHAPES = [(7, 5, 260), (9, 3, 12), (4, 6, 20), (3, 2, 4), (1, 1, 8), (13, 33, 64),
              (5, 7, 6), (3, 4, 130)]


@pytest.mark.parametrize("model", ["ac", "coupled"])
@pytest.mark.parametrize("shape", VEC_SHAPES)
def test_vector_kernels_match_oracle(model, shape):
    """FP64 runs on the vector stage kernels (two cells per thread) where n1
    is even; rows longer than a wavefront exercise the LDS neighbour reads."""
    for trial, faces in enumerate((0, 63, 1 | 2)):
        p, mask, phi, T = rand_problem(shape, model, 70 + trial, faces=faces, bc_kind=trial % 3)
        P = oracle.make_params(p)
        kp, kT = oracle.rhs(P, mask, 0.4, phi, T if model == "coupled" else None)
        from test_gpu_parity import gpu_rhs
        gp, gT = gpu_rhs(p, mask, 0.4, phi, T)
        assert rel(gp, kp) <= 1e-12
        if model == "coupled":
            assert rel(gT, kT) <= 1e-12
        dt = 2e-3 if model == "coupled" else 0.5
        ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt, phi,
                                        T if model == "coupled" else None, max_steps=3)
        for sched in ("five", "paired"):
            ph, th, st, d, cfg = run(p, mask, phi, T, dt, 3, "fp64", sched)
            assert rel(ph, ph_o) <= 1e-12, sched
            if model == "coupled":
                assert rel(th, T_o - T_STAR) <= 1e-12, sched


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vector_equals_one_cell(precision):
    p, mask, phi, T = rand_problem((21, 19, 260), "coupled", 12, faces=1 << 4, bc_kind=1)
    outs = []
    for vec in (True, False):
        s = pf.Solver(p, mask, precision, dict(tol=0.0))
        s.set_schedule("five")
        s.set_vector(vec)
        npdt = np.float64 if precision == "fp64" else np.float32
        s.set_state(phi.astype(npdt), (T - T_STAR).astype(npdt))
        s.set_time(0.0, 2e-3)
        s.integrate(max_steps=8)
        outs.append(s.get_state())
        s.close()
    tol = 1e-13 if precision == "fp64" else 2e-6
    assert rel(outs[0][0], outs[1][0]) <= tol and rel(outs[0][1], outs[1][1]) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotuned_stage_depths_do_not_change_results(precision):
    """The autotuner picks the planes per workgroup column of each stage pass
    separately; an adaptive run on its choice is bitwise equal to a run with
    one depth fixed for all passes (the per-cell arithmetic does not depend on
    the tiling, and the step-control reductions are maxima)."""
    p, mask, phi, T = rand_problem((40, 24, 36), "coupled", 31, faces=1 << 4, bc_kind=1)
    npdt = np.float64 if precision == "fp64" else np.float32
    outs = []
    for fixed in (None, 3):
        s = pf.Solver(p, mask, precision, dict(tol=1e-6))
        if fixed:
            s.set_tile(fixed)
        s.set_state(phi.astype(npdt), (T - T_STAR).astype(npdt))
        s.set_time(0.0, 1e-3)
        st = s.integrate(max_steps=40)
        cfg = s.get_config()
        outs.append((s.get_state(), st["steps_accepted"], st["steps_rejected"], cfg))
        s.close()
    (a, na, ra, cfg_a), (b, nb, rb, cfg_b) = outs
    assert all(1 <= z <= 40 for z in cfg_a["stage_z_chunk"]), cfg_a
    assert cfg_b["stage_z_chunk"] == [3] * 5, cfg_b
    assert (na, ra) == (nb, rb)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("precision,n1", [("fp64", 800), ("fp32", 1604)])
def test_rows_too_long_for_vector_lds(precision, n1):
    """Rows whose vector plane buffers would exceed 64 KiB of LDS run on the
    one-cell kernels: pf_set_vector(1) is refused, and the run still matches
    the oracle."""
    p, mask, phi, T = rand_problem((3, 2, n1), "coupled", 77, faces=1 << 4, bc_kind=1)
    s = pf.Solver(p, mask, precision, dict(tol=0.0))
    with pytest.raises(pf.PFError):
        s.set_vector(True)
    assert not s.get_config()["vector"]
    s.close()
    dt = 2e-3
    ph, th, st, d, cfg = run(p, mask, phi, T, dt, 3, precision, "five")
    assert not cfg["vector"]
    P = oracle.make_params(p)
    ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt, phi, T,
                                    max_steps=3)
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert rel(ph, ph_o) <= tol and rel(th, T_o - T_STAR) <= tol


def test_autotune_choice_is_reused_by_equal_handles():
    """A second handle of the same signature takes the first handle's
    autotuned configuration (no second measurement) and computes the same
    states."""
    p, mask, phi, T = rand_problem((24, 20, 32), "coupled", 91, faces=1 << 4, bc_kind=1)
    outs = []
    for rep in range(2):
        s = pf.Solver(p, mask, "fp32", dict(tol=1e-6))
        s.set_state(phi.astype(np.float32), (T - T_STAR).astype(np.float32))
        s.set_time(0.0, 1e-3)
        st = s.integrate(max_steps=30)
        outs.append((s.get_config(), s.get_state(), st["steps_accepted"]))
        s.close()
    assert outs[0][0] == outs[1][0]
    assert outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][1][0], outs[1][1][0])


@pytest.mark.parametrize("model", ["ac", "coupled"])
@pytest.mark.parametrize("shape", [(5, 3, 600), (4, 2, 1024), (2, 9, 12)])
def test_vector_fp32_depths_and_wide_rows(model, shape):
    """FP32 vector passes where the two halo rows exceed one vector per
    thread (n1 = 600, 1024: halo rows loaded in the plane they serve) and on a
    two-plane grid, at several planes per column (1, 2, 3 and the whole
    height: the plane-ahead loads stop at every column end): every depth gives
    the same state bitwise, equal to the one-cell kernels' within FP32
    rounding and to the oracle within the FP32 bound."""
    p, mask, phi, T = rand_problem(shape, model, 91, faces=1 << 4, bc_kind=1)
    dt = 2e-3 if model == "coupled" else 0.5
    coupled = model == "coupled"
    outs = []
    for vec, z in [(True, 1), (True, 2), (True, 3), (True, shape[0]), (False, 2)]:
        s = pf.Solver(p, mask, "fp32", dict(tol=0.0))
        s.set_schedule("five")
        s.set_vector(vec)
        s.set_tile(z)
        s.set_state(phi.astype(np.float32), (T - T_STAR).astype(np.float32) if coupled else None)
        s.set_time(0.0, dt)
        st = s.integrate(max_steps=4)
        assert st["steps_accepted"] == 4
        cfg = s.get_config()
        assert cfg["vector"] == vec and cfg["stage_z_chunk"] == [min(z, shape[0])] * 5, cfg
        outs.append(s.get_state())
        s.close()
    for o in outs[1:4]:
        assert np.array_equal(o[0], outs[0][0])
        if coupled:
            assert np.array_equal(o[1], outs[0][1])
    assert rel(outs[0][0], outs[4][0]) <= 2e-6
    P = oracle.make_params(p)
    ph_o, T_o, _ = oracle.integrate(P, mask, oracle.make_ctl(tol=0.0), 0.0, dt, phi,
                                    T if coupled else None, max_steps=4)
    assert rel(outs[0][0], ph_o) <= 1e-4
    if coupled:
        assert rel(outs[0][1], T_o - T_STAR) <= 1e-4
