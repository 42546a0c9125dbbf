"""Adjoint of the step: gradients of time-averaged channel objectives with
respect to (F_b, tau, A_1..A_M) against central finite differences of the
FP64 oracle, checkpoint-interval invariance, and the autograd wrapper."""
import numpy as np
import pytest

from oracle import geometry, objective
from paper_2205_04658_amd import workloads
from rlbtest import need_gpu

pytestmark = pytest.mark.gpu

NX, NY, TAU, FB, N = 64, 32, 0.8, 1e-4, 60
DISCS = np.array([[20.0, 16.0, 4.0], [45.5, 10.0, 3.0]])
MODES = workloads.stirring_basis(NX, NY, nmodes=4, kmin=2.0, kmax=4.0, seed=7)
AMPS = np.array([5e-5, -3e-5, 4e-5, 2e-5])


def fields():
    return workloads.random_fields(NX, NY, seed=21, beta=0.01)


def solid():
    return geometry.channel_mask(NX, NY, DISCS)


def gpu_lattice():
    from paper_2205_04658_amd.rlb import Lattice
    lat = Lattice(NX, NY, TAU, walls=True)
    f = fields()
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks(DISCS)
    return lat


@pytest.mark.parametrize("kind", ["current", "dissipation"])
def test_gradient_matches_oracle_finite_differences(kind):
    torch = need_gpu()
    lat = gpu_lattice()
    J, g = lat.adjoint_run(N, 7, kind, MODES, AMPS, FB)
    Jo = objective.run_objective(fields(), N, TAU, FB, MODES, AMPS, kind, solid())
    assert abs(J - Jo) <= 1e-4 * abs(Jo), (J, Jo)
    fd = objective.fd_gradient(fields(), N, TAU, FB, MODES, AMPS, kind, solid(), rel=1e-4)
    big = np.abs(fd) > 1e-2 * np.abs(fd).max()
    rel = np.abs(g - fd) / np.abs(fd)
    assert np.all(rel[big] < 2e-3), (g, fd)
    assert np.all(np.abs(g - fd)[~big] < 2e-3 * np.abs(fd).max()), (g, fd)


def test_checkpoint_interval_does_not_change_gradient():
    torch = need_gpu()
    out = []
    for K in (1, 7, 60, 100):
        lat = gpu_lattice()
        out.append(lat.adjoint_run(N, K, "current", MODES, AMPS, FB))
    for J, g in out[1:]:
        assert J == out[0][0]
        np.testing.assert_array_equal(g, out[0][1])


def test_forward_only_matches_and_advances():
    torch = need_gpu()
    lat = gpu_lattice()
    J0, g = lat.adjoint_run(N, 10, "current", MODES, AMPS, FB, grad=False)
    assert g is None and lat.step_count == N
    lat2 = gpu_lattice()
    J1, _ = lat2.adjoint_run(N, 10, "current", MODES, AMPS, FB)
    assert J0 == J1


def test_autograd_function():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import rlb_objective
    lat = gpu_lattice()
    theta = torch.tensor([FB, TAU, *AMPS], dtype=torch.float64, requires_grad=True)
    J = rlb_objective(theta, lat, fields(), MODES, N, 7, "current")
    J.backward()
    lat2 = gpu_lattice()
    Jr, gr = lat2.adjoint_run(N, 7, "current", MODES, AMPS, FB)
    assert float(J) == Jr
    np.testing.assert_array_equal(theta.grad.numpy(), gr)


def test_eta_s_relaxation_is_rejected_by_the_adjoint():
    """The adjoint differentiates a constant tau; a lattice relaxing with
    per-node tau from eta/s is refused (and accepted again after a constant
    tau is set), and batch members cannot set their own relaxation."""
    need_gpu()
    from paper_2205_04658_amd.rlb import Batch, EINVAL, EUNSUPPORTED, RLBError
    lat = gpu_lattice()
    lat.set_relaxation_eta_s(0.02, 0.05)
    with pytest.raises(RLBError) as e:
        lat.adjoint_run(N, 10, "current", MODES, AMPS, FB)
    assert e.value.status == EUNSUPPORTED
    with pytest.raises(RLBError) as e:
        lat.set_relaxation_eta_s(0.0, 0.05)
    assert e.value.status == EINVAL
    lat.set_relaxation_time(TAU)
    J, g = lat.adjoint_run(N, 10, "current", MODES, AMPS, FB)
    assert np.isfinite(J) and np.all(np.isfinite(g))
    B = Batch([(64, 16), (80, 24)], 0.8)
    for call in (lambda: B[0].set_relaxation_eta_s(0.02, 0.05), lambda: B[1].set_relaxation_time(0.9)):
        with pytest.raises(RLBError) as e:
            call()
        assert e.value.status == EINVAL
    B.close()
