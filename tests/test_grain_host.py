"""Host side of the grain batches (no GPU): the cost tables of the C ABI and
the argument checks that run before any device work."""
import ctypes

import numpy as np
import pytest

from paper_1602_05510_amd import hesp as H
from paper_1602_05510_amd import inputs as I
from oracle import oracle as O

PF = I.make_platform(I.cpu_accel_types(3, 2), seed=8)


def test_power_of_two_grain_tables_are_the_depth_tables():
    cost, xfer = H.cost_tables(PF.rmax, PF.h, 1024, 2)
    gcost, gxfer = H.grain_cost_tables(PF.rmax, PF.h, 1024, [1, 2, 4])
    assert np.array_equal(cost, gcost) and np.array_equal(xfer, gxfer)


def test_divisible_sides_match_the_oracle_task_time():
    fac, b = [1, 2, 3, 4, 6], 1536
    cost, xfer = H.grain_cost_tables(PF.rmax, PF.h, b, fac)
    for pt in range(PF.n_ptypes):
        for ty in range(4):
            for g, f in enumerate(fac):
                assert cost[pt, ty, g] == O.task_time(ty, b // f, int(PF.rmax[pt, ty]), int(PF.h[pt]))
    assert xfer.shape == (145,) and xfer[0] == 0
    for k in (1, 7, 144):                      # atoms of side 128
        assert xfer[k] == O.transfer_time(k, 128, PF)


def test_fractional_sides_round_up_once():
    # side 1024/3: the whole tile (9 atoms of L = 3) moves like one 1024-block
    _, xfer3 = H.grain_cost_tables(PF.rmax, PF.h, 1024, [1, 3])
    _, xfer1 = H.cost_tables(PF.rmax, PF.h, 1024, 0)
    assert xfer3[9] == xfer1[1]
    assert all(xfer3[k] <= xfer3[k + 1] for k in range(9))


def test_workspace_and_refusals():
    one = H.grain_workspace_bytes(4, [1, 2, 3], 3, 1)
    assert one > 0 and H.grain_workspace_bytes(4, [1, 2, 3], 3, 8) > 7 * (one - 8 * 37 - 256)
    for fac in ([], [0], [7, 11], [1, 2, 3, 4, 5, 6, 7, 8, 9]):
        with pytest.raises(H.HespError):
            H.grain_workspace_bytes(4, fac, 3, 1)
    with pytest.raises(H.HespError):
        H.grain_workspace_bytes(50, [1, 2, 3, 4], 3, 1)       # nt * L = 600 > 512
    pf = H.grain_platform(PF, 1024, [1, 2, 3])
    fake = ctypes.c_void_p(256)                                # never dereferenced: refused first
    fa = np.array([1, 2, 3], np.int32)
    gb = H.GrainBatchC(4, 3, 3, fa.ctypes.data_as(ctypes.c_void_p), fake)
    L = H.lib()
    for pol, code in (((0, 2, 0), H.HESP_EUNSUPPORTED), ((0, 3, 0), H.HESP_EUNSUPPORTED),
                      ((0, 0, 0, 0, 1), H.HESP_EUNSUPPORTED), ((2, 0, 0), H.HESP_EUNSUPPORTED)):
        rc = L.hesp_simulate_grain_batch(ctypes.byref(pf.c), H.Policy(*pol), ctypes.byref(gb), fake, None, None,
                                         None, fake, 1 << 40, 16, None)
        assert rc == code, pol
    bad = H.grain_platform(PF, 1024, [1, 2])                   # tables for two grains, batch has three
    rc = L.hesp_simulate_grain_batch(ctypes.byref(bad.c), H.Policy(0, 0, 0), ctypes.byref(gb), fake, None, None,
                                     None, fake, 1 << 40, 16, None)
    assert rc == H.HESP_EINVAL
    rc = L.hesp_simulate_grain_batch(ctypes.byref(pf.c), H.Policy(0, 0, 0), ctypes.byref(gb), fake, None, None,
                                     None, fake, 1024, 16, None)
    assert rc == H.HESP_ECAPACITY                              # workspace too small


def test_binding_checks_tensors():
    torch = pytest.importorskip("torch")
    pf = H.grain_platform(PF, 1024, [1, 2])
    g = torch.zeros((4, 10), dtype=torch.uint8)
    ms = torch.zeros(4, dtype=torch.int64)
    for bad in (dict(grain=g[:, :9]), dict(grain=g.to(torch.int32)), dict(makespan=ms[:3]),
                dict(makespan=ms.to(torch.int32)), dict(ws=torch.zeros(16, dtype=torch.uint8))):
        kw = dict(grain=g, makespan=ms)
        kw.update(bad)
        grain, makespan = kw.pop("grain"), kw.pop("makespan")
        with pytest.raises(H.HespError):
            H.simulate_grain_batch(pf, 3, [1, 2], grain, makespan, slots=1, **kw)
