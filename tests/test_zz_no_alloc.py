"""The entry point that allocates nothing (rlb_record_current_noalloc):
bitwise the series and states of rlb_record_current with a workspace, on
two calls in a row (the second with a smaller lattice and fewer steps, so
the fixed scratch still holds the first call's rows), and rejection of a
lattice whose rows do not fit the scratch."""
import numpy as np
import pytest

from paper_2205_04658_amd import workloads
from rlbtest import need_gpu

pytestmark = pytest.mark.gpu


def channel(nx, ny, full26, discs):
    from paper_2205_04658_amd.rlb import Lattice
    f = workloads.random_fields(nx, ny, seed=17, beta=0.01)
    lat = Lattice(nx, ny, 0.7, full26=full26, open_x=True)
    lat.init_fields(f["eps"], f["bx"], f["by"], f["n"])
    lat.add_disks(np.array(discs, np.float64))
    lat.set_open_borders(0.05, 0.0, 0.1, 1.0)
    return lat


def test_noalloc_equals_workspace_entry_point():
    torch = need_gpu()
    cases = [  # (nx, ny, full26, discs, steps, column): 2048 steps fill the scratch once
        (1024, 256, False, [(128.0, 128.0, 6.58), (208.6, 165.6, 6.58)], 2600, 1022),
        (200, 96, True, [(50.0, 40.0, 5.0)], 45, 7),
    ]
    for nx, ny, full, discs, steps, x in cases:
        print(f"noalloc case {nx}x{ny} full26={full} steps={steps} x={x}", flush=True)
        a_lat = channel(nx, ny, full, discs)
        a = a_lat.record_current(steps, x, chunk=1000)
        b_lat = channel(nx, ny, full, discs)
        b = b_lat.record_current_noalloc(steps, x)
        torch.cuda.synchronize()
        assert b_lat.step_count == steps
        assert torch.equal(a, b)
        assert torch.equal(a_lat.save_state().cpu(), b_lat.save_state().cpu())
        assert a.std().item() > 0.0


def test_noalloc_rejects_rows_beyond_the_scratch():
    need_gpu()
    from paper_2205_04658_amd.rlb import ENOMEM, Lattice, RLBError
    lat = Lattice(4, 524289, 0.7)      # 524289 rows x 8 bytes > 4 MiB
    with pytest.raises(RLBError) as e:
        lat.record_current_noalloc(3, 1)
    assert e.value.status == ENOMEM
    assert lat.step_count == 0
