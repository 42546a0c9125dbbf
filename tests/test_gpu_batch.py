"""Batched lattices (one launch per step over many lattices, hipGraph replay)
and launch shapes: every member evolves bitwise as the same lattice stepped
alone, for every launch shape, with or without graphs."""
import numpy as np
import pytest

from paper_2205_04658_amd import workloads
from rlbtest import need_gpu

pytestmark = pytest.mark.gpu

SIZES = [(70, 40), (128, 64), (65, 33), (200, 19)]
TAU = 0.8
FB = (2e-4, 0.0)


def setup_member(lat, b, nx, ny):
    f = workloads.random_fields(nx, ny, seed=100 + b, beta=0.02)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    discs = workloads.channel_discs(nx, ny, 4.0, 0.05, seed=7, stream=b)
    lat.add_disks(discs)


def single_runs(steps, shape=None):
    from paper_2205_04658_amd.rlb import Lattice
    out = []
    for b, (nx, ny) in enumerate(SIZES):
        lat = Lattice(nx, ny, TAU, walls=True)
        if shape:
            lat.set_launch_shape(*shape)
        setup_member(lat, b, nx, ny)
        lat.set_body_force(*FB)
        lat.step(steps)
        lat.sync()
        f, g = lat.planes()
        out.append((f.cpu(), g.cpu()))
    return out


def make_batch():
    from paper_2205_04658_amd.rlb import Batch
    B = Batch(SIZES, TAU, walls=True)
    for b, (nx, ny) in enumerate(SIZES):
        setup_member(B[b], b, nx, ny)
    B.set_body_force(*FB)
    return B


def test_launch_shapes_are_bitwise_identical():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    ref = None
    # 200 columns = 4 tiles per row: strips of 1, 3 (3 + a ragged 1) and 16
    for ty in (1, 2, 4, 8):
        for g in (0, 8):
            for sw in (1, 3, 16):
                lat = Lattice(200, 37, 0.7, walls=True)
                lat.set_launch_shape(ty, g, sw)
                assert lat.launch_shape() == (ty, g, sw)
                f = workloads.random_fields(200, 37, seed=4)
                lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
                lat.add_disks([(20.0, 15.0, 5.0), (150.0, 20.0, 4.0)])
                lat.set_stirring(2, 5, 1e-4, 9)
                lat.set_body_force(1e-4, 0)
                lat.step(11)
                s = lat.save_state().cpu()
                if ref is None:
                    ref = s
                assert torch.equal(s, ref), (ty, g, sw)


def test_tile_heights_the_layouts_support():
    """Tile heights 1, 2, 4, 8 for the folded set; 2 and 4 for the full set
    (its plain step is compiled for both); 4 for the planar set.  A
    refused shape leaves the current one."""
    need_gpu()
    from paper_2205_04658_amd.rlb import EUNSUPPORTED, Lattice, RLBError
    for kw, ok in ((dict(full26=True), (2, 4)), (dict(planar=True), (4,))):
        lat = Lattice(64, 16, 0.7, **kw)
        for ty in (1, 2, 8):
            lat.set_launch_shape(4, 4, 8)
            if ty in ok:
                lat.set_launch_shape(ty, 0, 16)
                assert lat.launch_shape() == (ty, 0, 16)
            else:
                with pytest.raises(RLBError) as e:
                    lat.set_launch_shape(ty, 0, 16)
                assert e.value.status == EUNSUPPORTED
                assert lat.launch_shape() == (4, 4, 8)


def test_full_set_tile_heights_are_bitwise_identical():
    """The full set's plain step at 2- and 4-row tiles, every grid and strip
    form, walls + discs + stirring + body force, and the field read-out
    (always 4-row tiles) after it."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Lattice
    ref = None
    for ty in (2, 4):
        for g in (0, 8):
            for sw in (1, 3, 16):
                lat = Lattice(200, 37, 0.7, walls=True, full26=True)
                lat.set_launch_shape(ty, g, sw)
                f = workloads.random_fields(200, 37, seed=4)
                lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
                lat.add_disks([(20.0, 15.0, 5.0), (150.0, 20.0, 4.0)])
                lat.set_stirring(2, 5, 1e-4, 9)
                lat.set_body_force(1e-4, 0)
                lat.step(11)
                s = lat.save_state().cpu()
                fl = lat.fields()["eps"].cpu()
                if ref is None:
                    ref = (s, fl)
                assert torch.equal(s, ref[0]), (ty, g, sw)
                assert torch.equal(fl, ref[1]), (ty, g, sw)


@pytest.mark.parametrize("graph", [16, 0], ids=["graph", "direct"])
def test_batch_members_equal_single_runs(graph):
    torch = need_gpu()
    steps = 37
    want = single_runs(steps)
    B = make_batch()
    B.use_graph(graph)
    B.step(steps)
    B.sync()
    for b in range(len(SIZES)):
        f, g = B[b].planes()
        assert torch.equal(f.cpu(), want[b][0]), b
        assert torch.equal(g.cpu(), want[b][1]), b
        assert B[b].step_count == steps


def test_graph_replays_with_eager_work_between():
    torch = need_gpu()
    want = single_runs(16 * 3 + 5)
    B = make_batch()
    B.step(5)                   # direct steps, odd phase
    for _ in range(3):          # three replays of one 16-step graph
        B.step(16)
        B[0].fields(["eps"])     # eager work between replays
        B[1].conserved()
    B.sync()
    for b in range(len(SIZES)):
        f, g = B[b].planes()
        assert torch.equal(f.cpu(), want[b][0]), b
        assert torch.equal(g.cpu(), want[b][1]), b


OPEN_SIZES = [(96, 40), (130, 33), (64, 24)]
OPEN_BORDERS = (0.06, 0.0, 0.12, 1.02)


def open_member(lat, b, nx, ny):
    f = workloads.random_fields(nx, ny, seed=200 + b, beta=0.01)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks([(nx / 3.0, ny / 2.0 - 0.5, 4.0 + b)])


@pytest.mark.parametrize("graph", [8, 0], ids=["graph", "direct"])
def test_open_channel_batch_equals_single_runs(graph):
    """A batch of Part II-like channels (one impurity placement per member,
    shared borders and body force) evolves bitwise as each channel alone,
    including a border change between runs."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Batch, Lattice
    want = []
    for b, (nx, ny) in enumerate(OPEN_SIZES):
        lat = Lattice(nx, ny, TAU, walls=True, open_x=True)
        open_member(lat, b, nx, ny)
        lat.set_open_borders(*OPEN_BORDERS)
        lat.set_body_force(*FB)
        lat.step(21)
        lat.set_open_borders(0.08, 0.01, 0.1, 1.0)
        lat.step(19)
        lat.sync()
        want.append(lat.save_state().cpu())
    B = Batch(OPEN_SIZES, TAU, walls=True, open_x=True)
    for b, (nx, ny) in enumerate(OPEN_SIZES):
        open_member(B[b], b, nx, ny)
    B.set_open_borders(*OPEN_BORDERS)
    B.set_body_force(*FB)
    B.use_graph(graph)
    B.step(21)
    B[0].fields(["eps"])
    B.set_open_borders(0.08, 0.01, 0.1, 1.0)
    B.step(19)
    B.sync()
    for b in range(len(OPEN_SIZES)):
        assert torch.equal(B[b].save_state().cpu(), want[b]), b


def test_member_rejects_settings_the_batch_holds():
    need_gpu()
    from paper_2205_04658_amd.rlb import EINVAL, RLBError
    B = make_batch()
    m = B[1]
    calls = [lambda: m.step(1), lambda: m.set_body_force(1e-4), lambda: m.set_stirring(1, 3, 1e-4, 1),
             lambda: m.set_relaxation_time(0.7), lambda: m.set_relaxation_eta_s(0.05, 0.05),
             lambda: m.set_launch_shape(2, 0, 16), lambda: m.autotune(1), lambda: m.use_graph(8),
             lambda: m.timing(True), lambda: m.record_current(2, 3)]
    for c in calls:
        with pytest.raises(RLBError) as e:
            c()
        assert e.value.status == EINVAL
    assert m.step_count == 0


def test_autotune_does_not_advance_and_keeps_results():
    torch = need_gpu()
    B = make_batch()
    B.step(3)
    before = [B[b].save_state().cpu() for b in range(len(SIZES))]
    rows = B.autotune(trials=2)
    assert len(rows) == 32 and all(r[3] > 0 for r in rows)
    after = [B[b].save_state().cpu() for b in range(len(SIZES))]
    for x, y in zip(before, after):
        assert torch.equal(x, y)
    B.step(34)
    want = single_runs(37)
    for b in range(len(SIZES)):
        f, g = B[b].planes()
        assert torch.equal(f.cpu(), want[b][0]), b


def test_member_cannot_step_alone():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import RLBError, EINVAL
    B = make_batch()
    with pytest.raises(RLBError) as e:
        B[0].step(1)
    assert e.value.status == EINVAL


REC_SIZES = [(96, 40), (130, 33), (64, 24)]
REC_BORDERS = (0.06, 0.01, 0.12, 1.05)


def rec_member(lat, b, nx, ny):
    f = workloads.random_fields(nx, ny, seed=300 + b, beta=0.01)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks([(nx / 4.0, ny / 2.0 - 0.5, 4.5)])
    return f


@pytest.mark.parametrize("x,chunk,full", [(-2, 1024, False), (0, 7, False), (3, 1, False),
                                          (-2, 7, True)])
def test_batch_record_current(x, chunk, full):
    """Open channels record in the step kernel: each member's series is
    bitwise the series of the same channel recorded alone, in chunks of
    1024, 7 and 1 steps (x < 0 counts from each member's outlet); it
    equals the column-current kernel on the same states up to float32
    sums in another order; the states match bitwise; member 0's series
    follows the FP64 oracle (j scale: n_in * beta_in); folded and full
    sets."""
    torch = need_gpu()
    from oracle import diagnostics, geometry, rlb as orl
    from paper_2205_04658_amd.rlb import Batch, Lattice
    steps = 25
    B = Batch(REC_SIZES, 0.7, open_x=True, full26=full)
    fs = [rec_member(B[b], b, nx, ny) for b, (nx, ny) in enumerate(REC_SIZES)]
    B.set_open_borders(*REC_BORDERS)
    B.step(3)
    got = B.record_current(steps, x, chunk=chunk)
    B.sync()
    assert got.shape == (len(REC_SIZES), steps)
    got = got.cpu()
    scale = 0.12 * 0.06
    for b, (nx, ny) in enumerate(REC_SIZES):
        def alone():
            lat = Lattice(nx, ny, 0.7, open_x=True, full26=full)
            rec_member(lat, b, nx, ny)
            lat.set_open_borders(*REC_BORDERS)
            lat.step(3)
            return lat
        lat = alone()
        want = lat.record_current(steps, x % nx).cpu()
        assert torch.equal(got[b], want), b
        assert torch.equal(B[b].save_state().cpu(), lat.save_state().cpu()), b
        lat = alone()
        col = torch.zeros(steps, dtype=torch.float64, device="cuda")
        for t in range(steps):
            lat.column_current(x % nx, out=col[t:t + 1])
            lat.step(1)
        assert (got[b] - col.cpu()).abs().max().item() < 1e-7 * scale, b
    nx, ny = REC_SIZES[0]
    solid = geometry.disc_mask(nx, ny, [(nx / 4.0, ny / 2.0 - 0.5, 4.5)])
    f = fs[0]
    F, G = orl.initial_state(*(f[k].astype(np.float64) for k in ("eps", "bx", "by", "n")))
    ref = []
    for t in range(3 + steps):
        if t >= 3:
            ref.append(diagnostics.column_current(orl.fields(F, G, solid=solid), x % nx))
        F, G = orl.step(F, G, 0.7, solid=solid, open_x=REC_BORDERS)
    assert np.abs(got[0].numpy() - np.array(ref)).max() < 1e-5 * scale
    assert np.ptp(ref) > 1e-3 * scale


@pytest.mark.parametrize("full", [False, True], ids=["folded17", "full26"])
def test_batch_record_current_periodic(full):
    """Periodic batches with walls, discs and a body force record with one
    column launch before each step: bitwise the column kernel on each
    member stepped alone, states bitwise equal."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Batch, Lattice
    steps, x = 12, -5
    B = Batch(SIZES, TAU, walls=True, full26=full)
    for b, (nx, ny) in enumerate(SIZES):
        setup_member(B[b], b, nx, ny)
    B.set_body_force(*FB)
    got = B.record_current(steps, x, chunk=5).cpu()
    for b, (nx, ny) in enumerate(SIZES):
        lat = Lattice(nx, ny, TAU, walls=True, full26=full)
        setup_member(lat, b, nx, ny)
        lat.set_body_force(*FB)
        want = torch.zeros(steps, dtype=torch.float64, device="cuda")
        for t in range(steps):
            lat.column_current(nx + x, out=want[t:t + 1])
            lat.step(1)
        assert torch.equal(got[b], want.cpu()), b
        assert torch.equal(B[b].save_state().cpu(), lat.save_state().cpu()), b
        assert got[b].std().item() > 0.0


def test_batch_record_current_errors_and_empty_runs():
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import EINVAL, EUNSUPPORTED, RLBError, Batch
    B = Batch(REC_SIZES, 0.7, open_x=True)
    for b, (nx, ny) in enumerate(REC_SIZES):
        rec_member(B[b], b, nx, ny)
    for x in (64, -65):                       # outside the 64-wide member
        with pytest.raises(RLBError) as e:
            B.record_current(2, x)
        assert e.value.status == EINVAL
    out = torch.empty((len(REC_SIZES), 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        B.record_current(5, -2, out=out)        # too short
    assert B.record_current(0, -2).shape == (len(REC_SIZES), 0)
    assert B.info()["step"] == 0
    wide = torch.full((len(REC_SIZES), 10), -1.0, dtype=torch.float64, device="cuda")
    B.record_current(4, 1, out=wide)            # row stride 10, first 4 columns written
    B.sync()
    w = wide.cpu()
    assert bool((w[:, 4:] == -1.0).all()) and bool((w[:, :4] != -1.0).all())
    assert B.info()["step"] == 4
    C = Batch([(64, 8), (70, 8)], 0.7, cfl=1.25)
    with pytest.raises(RLBError) as e:
        C.record_current(2, 1)
    assert e.value.status == EUNSUPPORTED


@pytest.mark.parametrize("graph", [16, 0], ids=["graph", "direct"])
def test_store_kind_does_not_change_results(graph):
    """The step kernels store with plain stores when a launch's two state
    copies fit in 224 MiB and with non-temporal stores above that: a batch
    holding a 1024^2 member (285 MB of state, non-temporal) advances its
    small members bit for bit as the same lattices stepped alone (plain).
    The 1024^2 member makes a group of its own, so the batch steps two
    groups in turn. One step first leaves the batch on its second state
    copy; the next 24 steps then take one step to realign, a 16-step graph
    and 7 direct steps group by group, or 24 direct steps group by group
    starting from the second copy."""
    torch = need_gpu()
    from paper_2205_04658_amd.rlb import Batch
    sizes = [(1024, 1024)] + SIZES[:2]
    B = Batch(sizes, TAU, walls=True)
    B.use_graph(graph)
    big = workloads.uniform(1024, 1024)
    B[0].init_fields(big["eps"], big["bx"], big["by"], big["n"])
    for b, (nx, ny) in enumerate(SIZES[:2]):
        setup_member(B[b + 1], b, nx, ny)
    B.set_body_force(*FB)
    B.step(1)
    B.step(24)
    B.sync()
    ref = single_runs(25)
    for b in range(3):
        assert B[b].step_count == 25, b
    for b in range(2):
        f, g = B[b + 1].planes()
        assert torch.equal(f.cpu(), ref[b][0]) and torch.equal(g.cpu(), ref[b][1]), b
    from paper_2205_04658_amd.rlb import Lattice
    lat = Lattice(1024, 1024, TAU, walls=True)
    lat.init_fields(big["eps"], big["bx"], big["by"], big["n"])
    lat.set_body_force(*FB)
    lat.step(25)
    lat.sync()
    f, g = B[0].planes()
    f1, g1 = lat.planes()
    assert torch.equal(f, f1) and torch.equal(g, g1)
