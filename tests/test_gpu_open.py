"""Open x borders (velocity inlet, pressure outlet) and the current-density
diagnostics on the GPU against the FP64 oracle: fields after a channel run
with an impurity (borders set inside the step kernel, or by a kernel of
their own when the outlet column starts a 64-node tile), the j(t) series at
the column before the outlet and its spectrum, plug flow in an empty
channel, launch shapes, and the error paths."""
import numpy as np
import pytest

from oracle import diagnostics, geometry, rlb
from paper_2205_04658_amd import workloads
from rlbtest import compare, need_gpu, scales

pytestmark = pytest.mark.gpu

TOL = 1e-5
NX, NY, TAU = 96, 40, 0.7
DISC = [(24.0, 19.5, 4.5)]
BORDERS = (0.06, 0.01, 0.12, 1.05)   # inlet beta_x, beta_y, n_in; outlet eps


def lattice(full26=False, cfl=1.0):
    from paper_2205_04658_amd.rlb import Lattice
    f = workloads.random_fields(NX, NY, seed=13, beta=0.01)
    lat = Lattice(NX, NY, TAU, cfl=cfl, full26=full26, open_x=True)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks(np.array(DISC))
    lat.set_open_borders(*BORDERS)
    return lat, f


def oracle_start(f):
    return rlb.initial_state(*(f[k].astype(np.float64) for k in ("eps", "bx", "by", "n")))


@pytest.mark.parametrize("full", [False, True], ids=["folded17", "full26"])
@pytest.mark.parametrize("cfl", [1.0, 0.5])
def test_open_channel_parity(full, cfl):
    torch = need_gpu()
    lat, f = lattice(full, cfl)
    steps = 60
    lat.step(steps)
    lat.sync()
    solid = geometry.disc_mask(NX, NY, DISC)
    F, G = oracle_start(f)
    for _ in range(steps):
        F, G = rlb.step(F, G, TAU, cfl=cfl, solid=solid, open_x=BORDERS)
    err = compare(lat.fields(), rlb.fields(F, G, cfl=cfl, solid=solid), scales(beta=0.06, n=0.12))
    assert max(err.values()) < TOL, err


@pytest.mark.parametrize("nx", [64, 129, 190])
def test_open_channel_widths(nx):
    """64: both borders in one tile; 129 = 2 * 64 + 1: the outlet column
    starts a tile (separate border kernel); 190: ragged last tile."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    ny, steps = 24, 40
    disc = [(nx / 3, 11.5, 3.5)]
    f = workloads.random_fields(nx, ny, seed=31, beta=0.01)
    lat = Lattice(nx, ny, TAU, walls=True, open_x=True)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks(np.array(disc))
    lat.set_open_borders(*BORDERS)
    lat.set_body_force(2e-5, 0.0)
    lat.step(steps)
    solid = geometry.channel_mask(nx, ny, disc)
    F, G = oracle_start(f)
    force = np.zeros((3, ny, nx))
    force[0] = 2e-5
    for _ in range(steps):
        F, G = rlb.step(F, G, TAU, solid=solid, open_x=BORDERS, force=force)
    err = compare(lat.fields(), rlb.fields(F, G, solid=solid), scales(beta=0.06, n=0.12))
    assert max(err.values()) < TOL, err


def test_open_launch_shapes_are_bitwise_identical():
    torch = need_gpu()
    ref = None
    for shape in [(1, 0, 4), (2, 0, 16), (4, 4, 8), (8, 0, 1)]:
        lat, _ = lattice()
        lat.set_launch_shape(*shape)
        lat.set_stirring(2, 4, 1e-4, 3)
        lat.step(17)
        s = lat.save_state().cpu()
        if ref is None:
            ref = s
        assert torch.equal(s, ref), shape


def test_border_tiles_first_order():
    """256 x 64 channel, 1-row tiles: with a strip as wide as the lattice
    the border tiles run first within each XCD's share (eight whole tile
    rows each); with 1-tile strips the tiles keep the plain order.  Both
    give the same state bit for bit, and match the FP64 oracle."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    nx, ny, steps = 256, 64, 30
    disc = [(90.0, 30.5, 5.0)]
    f = workloads.random_fields(nx, ny, seed=41, beta=0.01)
    states = []
    # one workgroup per tile and a persistent grid (4 per CU), both in the
    # border-first order; then 1-tile strips (plain order)
    for shape in [(1, 0, 16), (1, 4, 16), (2, 4, 32), (1, 0, 1)]:
        lat = Lattice(nx, ny, TAU, open_x=True)
        lat.set_launch_shape(*shape)
        lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
        lat.add_disks(np.array(disc))
        lat.set_open_borders(*BORDERS)
        lat.step(steps)
        states.append(lat.save_state().cpu())
        if len(states) == 1:
            fields = lat.fields()
    for st in states[1:]:
        assert torch.equal(states[0], st)
    solid = geometry.disc_mask(nx, ny, disc)
    F, G = oracle_start(f)
    for _ in range(steps):
        F, G = rlb.step(F, G, TAU, solid=solid, open_x=BORDERS)
    err = compare(fields, rlb.fields(F, G, solid=solid), scales(beta=0.06, n=0.12))
    assert max(err.values()) < TOL, err


def test_current_series_and_spectrum():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import power_spectrum
    lat, f = lattice()
    steps, x = 64, NX - 2
    series = torch.zeros(steps, dtype=torch.float64, device="cuda")
    solid = geometry.disc_mask(NX, NY, DISC)
    F, G = oracle_start(f)
    want = []
    for t in range(steps):
        lat.step(1)
        lat.column_current(x, out=series[t:t + 1])
        F, G = rlb.step(F, G, TAU, solid=solid, open_x=BORDERS)
        want.append(diagnostics.column_current(rlb.fields(F, G, solid=solid), x))
    got = series.cpu().numpy()
    want = np.array(want)
    scale = 0.12 * 0.06
    assert np.abs(got - want).max() < TOL * scale
    assert np.ptp(want) > 1e-3 * scale          # the series does fluctuate
    p = power_spectrum(series).cpu().numpy()
    ref = diagnostics.power_spectrum(got)        # same input: only the sum order differs
    assert np.abs(p - ref).max() < 1e-12 * ref.max()
    ref_o = diagnostics.power_spectrum(want)     # oracle series
    assert np.abs(p - ref_o).max() < 1e-3 * ref_o.max()


@pytest.mark.parametrize("x,chunk,full", [(NX - 2, 1024, False), (0, 7, False),
                                          (int(DISC[0][0]), 1, False), (NX - 2, 7, True)])
def test_record_current_equals_sample_and_step(x, chunk, full):
    """The series the step kernel records equals the column-current kernel
    on the same states (float32 sums in another order), in chunks of 1024,
    7 (several chunks and a ragged one) and 1 steps, folded and full sets;
    the states match bitwise."""
    torch = need_gpu()
    steps = 30
    lat, _ = lattice(full)
    a = torch.zeros(steps, dtype=torch.float64, device="cuda")
    for t in range(steps):
        lat.column_current(x, out=a[t:t + 1])
        lat.step(1)
    lat2, _ = lattice(full)
    b = lat2.record_current(steps, x, chunk=chunk)
    assert lat2.step_count == steps
    assert torch.equal(lat.save_state().cpu(), lat2.save_state().cpu())
    scale = 0.12 * 0.06
    assert (a - b).abs().max().item() < 1e-7 * scale
    assert a.std().item() > 1e-5 * scale


@pytest.mark.parametrize("open_x,nx", [(False, 96), (True, 129)], ids=["periodic", "tile_edge"])
def test_record_current_without_fused_borders(open_x, nx):
    """Periodic folded lattices and widths with nx % 64 == 1 record with the
    column kernel before each step: bitwise the explicit loop."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice

    def make():
        f = workloads.random_fields(nx, 24, seed=5, beta=0.02)
        lat = Lattice(nx, 24, TAU, open_x=open_x)
        lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
        lat.set_body_force(1e-4, 0.0)
        return lat
    lat = make()
    a = torch.zeros(12, dtype=torch.float64, device="cuda")
    for t in range(12):
        lat.column_current(nx - 2, out=a[t:t + 1])
        lat.step(1)
    b = make().record_current(12, nx - 2, chunk=5)
    assert torch.equal(a, b)


def test_record_current_periodic_full_set():
    """Periodic lattices of the full set record in the step kernel."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice

    def make():
        f = workloads.random_fields(96, 24, seed=6, beta=0.02)
        lat = Lattice(96, 24, TAU, walls=True, full26=True)
        lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
        lat.add_disks(np.array([(50.0, 12.0, 4.0)]))
        lat.set_stirring(1, 3, 1e-4, 8)
        return lat
    lat = make()
    a = torch.zeros(20, dtype=torch.float64, device="cuda")
    for t in range(20):
        lat.column_current(50, out=a[t:t + 1])
        lat.step(1)
    lat2 = make()
    b = lat2.record_current(20, 50, chunk=6)
    assert torch.equal(lat.save_state().cpu(), lat2.save_state().cpu())
    scale = 0.1 * 0.02
    assert (a - b).abs().max().item() < 1e-7 * scale
    assert a.std().item() > 1e-5 * scale


def test_power_spectrum_of_a_cosine():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import power_spectrum
    n = 1000
    t = np.arange(n)
    s = 1.5 + 0.25 * np.cos(2 * np.pi * 37 * t / n + 0.4)
    p = power_spectrum(torch.tensor(s, device="cuda")).cpu().numpy()
    assert abs(p[37] - 0.25 ** 2 / 4) < 1e-14
    assert np.delete(p, 37).max() < 1e-24


def test_empty_channel_becomes_plug_flow():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    lat = Lattice(12, 4, 1.5, open_x=True)
    f = workloads.uniform(12, 4, eps=1.2, n=0.1)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.set_open_borders(0.1, 0.0, 0.15, 1.0)
    lat.step(4000)
    g = {k: v.cpu().numpy()[:, 2:-2] for k, v in lat.fields(["eps", "beta_x", "beta_y", "n"]).items()}
    assert np.abs(g["beta_x"] - 0.1).max() < 1e-5
    assert np.abs(g["beta_y"]).max() < 1e-6
    assert np.abs(g["eps"] - 1.0).max() < 1e-5
    assert np.abs(g["n"] - 0.15).max() < 1e-5


def test_open_border_errors():
    need_gpu()
    from paper_2205_04658_amd.rlb import Batch, EINVAL, EUNSUPPORTED, Lattice, RLBError
    periodic = Lattice(32, 8, 0.8)
    with pytest.raises(RLBError) as e:
        periodic.set_open_borders(0.1, 0.0, 0.1, 1.0)
    assert e.value.status == EINVAL
    lat = Lattice(32, 8, 0.8, open_x=True)
    for args in [(0.8, 0.7, 0.1, 1.0), (0.1, 0.0, np.nan, 1.0), (0.1, 0.0, 0.1, 0.0)]:
        with pytest.raises(RLBError) as e:
            lat.set_open_borders(*args)
        assert e.value.status == EINVAL
    with pytest.raises(RLBError) as e:
        lat.column_current(32)
    assert e.value.status == EINVAL
    with pytest.raises(RLBError) as e:
        lat.adjoint_run(4, 2, "current", np.zeros((0, 5)), np.zeros(0), 1e-6)
    assert e.value.status == EUNSUPPORTED
    with pytest.raises(RLBError) as e:
        Batch([(32, 8), (65, 8)], 0.8, open_x=True)       # 65 % 64 == 1
    assert e.value.status == EUNSUPPORTED
    B = Batch([(32, 8), (40, 8)], 0.8, open_x=True)
    with pytest.raises(RLBError) as e:
        B[1].set_open_borders(0.1, 0.0, 0.1, 1.0)          # members share the batch's
    assert e.value.status == EINVAL
    with pytest.raises(RLBError) as e:
        B.set_open_borders(1.1, 0.0, 0.1, 1.0)
    assert e.value.status == EINVAL
    with pytest.raises(RLBError) as e:
        Batch([(32, 8), (40, 8)], 0.8).set_open_borders(0.1, 0.0, 0.1, 1.0)
    assert e.value.status == EINVAL
