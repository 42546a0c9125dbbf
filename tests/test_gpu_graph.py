"""Graph replay of single lattices: a lattice stepped through HIP graphs
evolves bitwise as the same lattice stepped kernel by kernel, with eager
work between replays, parity alignment from the second state copy, graphs
recaptured after a setting changes, and timing (which bypasses graphs)."""
import numpy as np
import pytest

from paper_2205_04658_amd import workloads
from rlbtest import need_gpu

pytestmark = pytest.mark.gpu

K = 8


def stirred(nx=160, ny=72):
    from paper_2205_04658_amd.rlb import Lattice
    lat = Lattice(nx, ny, 0.75, walls=True)
    f = workloads.random_fields(nx, ny, seed=21, beta=0.02)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks([(40.0, 30.0, 6.0), (110.0, 45.0, 5.0)])
    lat.set_stirring(2, 6, 1e-4, 17)
    lat.set_body_force(1e-4, 0.0)
    return lat


def channel(nx=128, ny=48):
    from paper_2205_04658_amd.rlb import Lattice
    lat = Lattice(nx, ny, 0.7, open_x=True)
    f = workloads.random_fields(nx, ny, seed=22, beta=0.01)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks([(32.0, 23.5, 5.5)])
    lat.set_open_borders(0.05, 0.0, 0.1, 1.02)
    lat.set_relaxation_eta_s(0.05, 0.05)
    return lat


def drive(lat, graph, changes):
    """5 steps (odd phase), 2K + 1 (aligns, two replays), eager reads, K,
    then `changes` (a setting the graph holds by value) and 2K + 3."""
    lat.use_graph(graph)
    lat.step(5)
    lat.step(2 * K + 1)
    lat.fields(["eps", "beta_x"])
    lat.conserved()
    lat.step(K)
    lat.fields(["n"])
    changes(lat)
    lat.step(2 * K + 3)
    lat.sync()
    assert lat.step_count == 5 + 2 * K + 1 + K + 2 * K + 3
    return lat.save_state().cpu()


@pytest.mark.parametrize("make,change", [
    (stirred, lambda lat: lat.set_body_force(-5e-5, 2e-5)),
    (stirred, lambda lat: lat.set_stirring(1, 4, 2e-4, 5)),
    (channel, lambda lat: lat.set_open_borders(0.07, 0.01, 0.1, 1.0)),
    (channel, lambda lat: lat.set_relaxation_time(0.65)),
    (channel, lambda lat: lat.add_disks([(90.0, 10.0, 4.0)])),
], ids=["body_force", "stirring", "open_borders", "tau", "obstacle"])
def test_graph_equals_direct(make, change):
    torch = need_gpu()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        want = drive(make(), 0, change)
        got = drive(make(), K, change)
    assert torch.equal(got, want)


def test_timing_bypasses_graph_and_counts_every_step():
    torch = need_gpu()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        want = drive(stirred(), 0, lambda lat: None)
        lat = stirred()
        lat.timing(True)
        got = drive(lat, K, lambda lat: None)
        ms, n = lat.timing_read()
    assert torch.equal(got, want)
    assert n == 5 + 2 * K + 1 + K + 2 * K + 3 and ms > 0


def test_null_stream_runs_direct():
    torch = need_gpu()
    want = drive(stirred(), 0, lambda lat: None)
    got = drive(stirred(), K, lambda lat: None)
    assert torch.equal(got, want)


def test_use_graph_rejects_odd_and_negative_counts():
    need_gpu()
    from paper_2205_04658_amd.rlb import RLBError
    lat = stirred(64, 16)
    for bad in (-2, 3, 4098):
        with pytest.raises(RLBError):
            lat.use_graph(bad)
    lat.use_graph(0)
    lat.use_graph(4096)
