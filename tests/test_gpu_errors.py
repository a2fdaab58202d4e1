"""Error paths of the C ABI that need a solver (hence a GPU): every failure is
a status code with a message, never a crash, and the solver stays usable."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _pk():
    import paper_2609_09990_amd as pk
    return pk


def _solver(pk, **kw):
    h, B, e0 = synth.make_hamiltonian(6, 8, 0)
    return pk.Solver(pk.Problem(h, B, 3, 3, e0), **kw)


def test_step_away_from_the_centre_is_refused_then_sweep_works():
    pk = _pk()
    sol = _solver(pk, M=32, tol=1e-9)
    with pytest.raises(pk.DMRGError) as e:
        sol.step(3, 0)
    assert e.value.code == -6 and "orthogonality" in str(e.value)
    e0, tau, ok = sol.step(0, 0)
    assert ok
    e1, tau, ok = sol.sweep(1)
    assert ok and e1[0] <= e0[0] + 1e-9


def test_not_converged_fills_outputs_and_reports():
    pk = _pk()
    sol = _solver(pk, M=32, tol=1e-14, max_iter=2)
    e, tau, ok = sol.step(0, 0)
    assert not ok and np.isfinite(e[0])
    assert sol.stats()["converged"] == 0


def test_invalid_arguments():
    pk = _pk()
    sol = _solver(pk, M=16)
    with pytest.raises(pk.DMRGError) as e:
        sol.step(5, 0)  # k + 1 must be < n_orb
    assert e.value.code == -1
    with pytest.raises(pk.DMRGError) as e:
        sol.set_precond(1, None)  # learned without a network
    assert e.value.code == -1
    with pytest.raises(pk.DMRGError) as e:
        sol.set_precond(1, pk.MLP(5, 16))  # the preconditioner network takes 8 features
    assert e.value.code == -1
    with pytest.raises(pk.DMRGError) as e:
        _solver(pk, M=16, n_states=9)
    assert e.value.code == -1
    with pytest.raises(pk.DMRGError) as e:
        _solver(pk, M=16, n_states=2, weights=[1.0, -1.0])
    assert e.value.code == -1
    with pytest.raises(ValueError):
        sol.grad(np.ones(3))


def test_excited_state_gradient_needs_centre_tensors():
    pk = _pk()
    sol = _solver(pk, M=16, n_states=2)
    with pytest.raises(pk.DMRGError) as e:
        sol.grad(np.array([0.0, 1.0]))  # no sweep yet: only root 0 exists
    assert e.value.code == -6
    dh, dB, en = sol.grad(np.array([1.0, 0.0]))
    assert np.isfinite(dh).all() and abs(np.trace(dh) - 6.0) < 1e-10


def test_device_vector_lengths_are_checked():
    """Entry points that take device vectors check their length on the host
    (a wrong length is DMRG_EINVAL, nothing is launched): the CI calls against
    the CI dimension, the correction call against the two-site length."""
    import ctypes as C

    import torch
    pk = _pk()
    from paper_2609_09990_amd import _lib
    sol = _solver(pk, M=16)
    prob = sol.problem
    na, nb = prob.ci_dims()
    c = torch.zeros(na * nb + 1, dtype=torch.float64, device="cuda")
    g, G, o = np.zeros((6, 6)), np.zeros((6,) * 4), C.c_double()
    stream = torch.cuda.current_stream().cuda_stream
    assert _lib.dmrg_ci_rdm12(prob.h, na * nb + 1, _lib._ptr(c), _lib._ptr(c), _lib._ptr(g), _lib._ptr(G),
                              C.byref(o), stream) == -1
    assert _lib.dmrg_ci_apply_v(prob.h, na * nb - 1, _lib._ptr(c), _lib._ptr(c[1:]), stream) == -1
    with pytest.raises(ValueError):
        prob.ci_rdm12(c)  # the binding refuses the tensor before the call
    n = sol.prepare(2)
    x = torch.zeros(n + 3, dtype=torch.float64, device="cuda")
    mv = C.c_int()
    assert _lib.dmrg_correction(sol.h, 2, 0, n + 3, _lib._ptr(x), _lib._ptr(x), _lib._ptr(x), 0.0, _lib._ptr(x),
                                C.byref(mv)) == -1
    e, tau, ok = sol.sweep(1)  # still usable
    assert np.isfinite(e[0])
