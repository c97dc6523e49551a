"""The allocation-free gradient contraction (ns_resistance_gradient_noalloc)
against the workspace one (ns_resistance_gradient), through the C ABI: two
calls in a row on different contexts, the second with fewer outlets and
nodes, share the library's file-scope scratch; and the call captured into a
HIP graph, replayed with new inputs between replays."""
import ctypes as C

import numpy as np
import pytest
import torch

from conftest import get_case

pytestmark = pytest.mark.gpu


def _noalloc(ctx, lam, x, out, stream=None):
    st = C.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    p = [C.c_void_p(t.data_ptr() if t is not None else None) for t in (lam, x, out)]
    return ctx.lib.ns_resistance_gradient_noalloc(ctx.h, *p, st)


def _context(name, seed):
    from paper_1911_10814_amd import NsContext
    c = get_case(name)
    ctx = NsContext(c).bind()
    R = c.R * (1.0 + 0.5 * np.random.default_rng(seed).random(c.n_outlets))
    ctx.assemble(c.v, c.p, c.vdot, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, R=R)
    return ctx


def test_noalloc_gradient_matches_the_workspace_entry_point():
    results = []
    for name, seed in (("plate_small", 1), ("channel2", 2)):  # the second call has fewer outlets and nodes
        ctx = _context(name, seed)
        rng = np.random.default_rng(seed + 10)
        lam = torch.as_tensor(rng.standard_normal(4 * ctx.N), device="cuda")
        x = torch.as_tensor(rng.standard_normal(4 * ctx.N), device="cuda")
        ref = ctx.resistance_gradient(lam, x)
        out = torch.full((ctx.n_out,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(ctx, lam, x, out) == 0, ctx.lib.ns_last_error(ctx.h).decode()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), (name, got, ref)
        assert np.all(np.abs(got) > 0)
        results.append(got)
        ctx.close()
    assert len(results[0]) == 16 and len(results[1]) == 2


def test_noalloc_gradient_under_graph_capture_and_state_errors():
    ctx = _context("plate_small", 3)
    rng = np.random.default_rng(4)
    lam = torch.as_tensor(rng.standard_normal(4 * ctx.N), device="cuda")
    x = torch.as_tensor(rng.standard_normal(4 * ctx.N), device="cuda")
    out = torch.zeros(ctx.n_out, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # one eager call on the capture stream first
        assert _noalloc(ctx, lam, x, out, side) == 0
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        st = _noalloc(ctx, lam, x, out)
    assert st == 0
    for rep in range(3):
        lam.copy_(torch.as_tensor(rng.standard_normal(4 * ctx.N), device="cuda"))
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = ctx.resistance_gradient(lam, x)
        assert np.array_equal(out.cpu().numpy(), ref), rep
    # a tangent assembled from the reduced-model data leaves nothing to differentiate
    c = get_case("plate_small")
    ctx.assemble(c.v, c.p, c.vdot, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, m=c.R, P_af=c.R)
    assert _noalloc(ctx, lam, x, out) == -6
    assert b"resistance" in ctx.lib.ns_last_error(ctx.h)
    R = c.R * 1.1
    ctx.assemble(c.v, c.p, c.vdot, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, R=R)
    assert _noalloc(ctx, lam, None, out) == -1  # null pointer
    ctx.close()
