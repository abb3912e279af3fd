"""Stream arguments of the boundary: the state copies, the right-hand side and
the warm start issued on a caller stream give the same results as on the
handle's own stream."""
import numpy as np
import pytest

import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2401_01672_amd as pf  # noqa: E402

T_STAR = pi.T_STAR


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_caller_stream_rhs_and_state(precision):
    c = pi.crop_case(pi.case_coupled_128(), lo=(40, 40, 0), size=(24, 20, 18))
    dt = torch.float64 if precision == "fp64" else torch.float32
    npdt = np.float64 if precision == "fp64" else np.float32
    s = pf.Solver(c.params, c.mask, precision, dict(c.run, tol=0.0))
    rng = np.random.default_rng(3)
    phi = np.clip(c.phi0 + 0.3 * rng.random(c.phi0.shape), 0, 1).astype(npdt)
    th = (c.T0 - T_STAR + rng.normal(0, 0.5, c.T0.shape)).astype(npdt)
    ph_d = torch.tensor(phi, device="cuda")
    th_d = torch.tensor(th, device="cuda")
    ref_p, ref_t = torch.empty_like(ph_d), torch.empty_like(th_d)
    s.rhs(0.25, ph_d, th_d, ref_p, ref_t)  # the handle's stream
    side = torch.cuda.Stream()  # default priority
    got_p = torch.full_like(ph_d, float("nan"))
    got_t = torch.full_like(th_d, float("nan"))
    torch.cuda.synchronize()
    s.rhs(0.25, ph_d, th_d, got_p, got_t, stream=side.cuda_stream)
    side.synchronize()
    assert torch.equal(got_p, ref_p) and torch.equal(got_t, ref_t)
    # state copies on the caller stream
    s.set_state(ph_d, th_d, stream=side.cuda_stream)
    a, b = s.get_state(stream=side.cuda_stream)
    assert np.array_equal(a, phi) and np.array_equal(b, th)
    s.close()
