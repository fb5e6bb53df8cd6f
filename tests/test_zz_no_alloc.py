"""The allocation-free volume potential (nvp_volume_potential_noalloc) through the C ABI.

Its output is checked against nvp_volume_potential's on the same inputs, two
calls in a row with the second on a smaller grid (the fixed scratch keeps the
first call's contents), in both precisions, at the parity gates (relative L2
1e-12 complex128, 1e-5 complex64); the smaller case is also checked against
the oracle's direct midpoint sum.  The calls must leave the device's free
memory unchanged, and a grid beyond the fixed scratch is refused.
"""

import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from workload import fields

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2011_03009_amd")
from paper_2011_03009_amd import _native  # noqa: E402

TOL = {P.NVP_C64: 1e-5, P.NVP_C128: 1e-12}
DT = {P.NVP_C64: torch.complex64, P.NVP_C128: torch.complex128}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def noalloc(ctx, k, g, f, out):
    """Direct C-ABI call of the allocation-free entry point."""
    gg = P.grid(g)
    return _native.lib().nvp_volume_potential_noalloc(ctx.handle, k.real, k.imag, ctypes.byref(gg),
                                                      ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                      P.nvp.prec_of(f.dtype))


def rel(a, b):
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


@pytest.mark.parametrize("prec", [P.NVP_C64, P.NVP_C128])
def test_noalloc_matches_volume_potential_two_calls(prec):
    ctx = P.Context(0)
    try:
        k = complex(2 * 4647.91, 0.5)
        cases = [((40, 36, 50), 1.0e-4, 11), ((17, 23, 30), 7.5e-5, 12)]  # the second is smaller
        ins, refs = [], []
        for n, h, seed in cases:
            g = oracle.Grid((0.01, -0.002, 0.003), h, n)
            f = torch.from_numpy(fields.random_field(n, seed)).to("cuda").to(DT[prec])
            ins.append((g, f))
            refs.append(P.volume_potential(ctx, k, g, f))  # loads the kernels of these lengths
        torch.cuda.synchronize()
        outs = [torch.empty_like(f) for _, f in ins]
        free0 = torch.cuda.mem_get_info()[0]
        for (g, f), out in zip(ins, outs):
            say("case noalloc prec=%d n=%s" % (prec, g.n))
            assert noalloc(ctx, k, g, f, out) == 0, _native.lib().nvp_last_error(ctx.handle)
        ctx.sync()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 >= free0, (free0, free1)
        for out, ref in zip(outs, refs):
            e = rel(out, ref)
            say("  noalloc vs volume_potential rel L2 %.3e, bitwise %s" % (e, bool(torch.equal(out, ref))))
            assert e < TOL[prec]
        (g, f), out = ins[1], outs[1]
        want = -oracle.conv_direct(f.to(torch.complex128).cpu().numpy(), g.h, k)
        assert oracle.rel_l2(out.to(torch.complex128).cpu().numpy(), want) < TOL[prec]
    finally:
        ctx.close()


def test_noalloc_refuses_grids_beyond_the_scratch():
    ctx = P.Context(0)
    try:
        n = (200, 200, 200)  # its buffers exceed the fixed scratch; refused before any device work
        g = oracle.Grid((0.0, 0.0, 0.0), 1e-4, n)
        f = torch.zeros(n, dtype=torch.complex64, device="cuda")
        out = torch.empty_like(f)
        st = noalloc(ctx, complex(9000.0, 0.0), g, f, out)
        assert st == 4
        assert b"scratch" in _native.lib().nvp_last_error(ctx.handle)
        with pytest.raises(P.NvpError) as e:
            P.volume_potential_noalloc(ctx, 9000.0, g, f, out)
        assert e.value.status == 4
        # still usable afterwards
        small = oracle.Grid((0.0, 0.0, 0.0), 1e-4, (9, 10, 11))
        fs = torch.from_numpy(fields.random_field(small.n, 3)).to("cuda").to(torch.complex64)
        us = torch.empty_like(fs)
        P.volume_potential_noalloc(ctx, 9000.0 + 0.5j, small, fs, us)
        ref = -oracle.conv_direct(fs.to(torch.complex128).cpu().numpy(), small.h, 9000.0 + 0.5j)
        assert oracle.rel_l2(us.to(torch.complex128).cpu().numpy(), ref) < 1e-5
    finally:
        ctx.close()
