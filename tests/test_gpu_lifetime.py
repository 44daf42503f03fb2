"""Context lifetime through the C ABI: handles made from a context (cells,
ROMs, solutions, engines) may be freed before or after it, in any order --
the context's stream, allocator and pinned memory go with the last of them.
Exercised explicitly (the context closed first, a solution still read
afterwards) and through Python's cycle collector, which finalises a
context and its handles in an order of its own choosing."""
import gc

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SPEC = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 3), tsv_diameter=1.6)


@pytest.fixture(scope="module")
def mos():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos
    return mos


def make_all(mos):
    ctx = mos.Context(0)
    cell = mos.mos_build_cell(ctx, SPEC)
    rom = mos.mos_reduce(ctx, cell)
    sol = mos.mos_solve_array(ctx, [rom], 2, 2, np.zeros(4, dtype=np.uint8), -250.0)
    eng = mos.Engine(ctx, [rom], device_bytes=1 << 26)
    return ctx, cell, rom, sol, eng


def test_handles_outlive_their_context(mos):
    ctx, cell, rom, sol, eng = make_all(mos)
    u0, res0, it0 = mos.mos_get_solution(sol)
    ctx.close()
    u1, res1, it1 = mos.mos_get_solution(sol)
    assert np.array_equal(u0, u1) and res0 == res1 and it0 == it1
    for h in (cell, sol, eng, rom):
        h.close()


@pytest.mark.parametrize("order", ["ctx_first", "ctx_last", "mixed"])
def test_any_free_order(mos, order):
    ctx, cell, rom, sol, eng = make_all(mos)
    seq = {"ctx_first": (ctx, rom, eng, sol, cell), "ctx_last": (sol, eng, rom, cell, ctx),
           "mixed": (rom, ctx, sol, cell, eng)}[order]
    for h in seq:
        h.close()


def test_context_and_handles_collected_together(mos):
    for _ in range(4):
        objs = list(make_all(mos))
        objs.append(objs)            # a reference cycle: collected by the cycle collector
        del objs
        gc.collect()
    # The device and the library still work afterwards.
    ctx, cell, rom, sol, eng = make_all(mos)
    u, res, it = mos.mos_get_solution(sol)
    assert res <= 1e-12 and np.isfinite(u).all()
