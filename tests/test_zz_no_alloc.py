"""pbfb_residual_noalloc (the residual for callers that cannot allocate) against
pbfb_residual through the C ABI: two calls in a row, the second on a smaller
problem, each equal to the allocating entry point's result (same kernels, so
bit for bit) and to the oracle within the FP64 bar; the error paths (not set
up, host memory, a problem too large for the fixed work array)."""
import numpy as np
import pytest

import oracle
import pbgen
from conftest import cached_config

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def test_noalloc_residual_matches_the_allocating_one():
    import torch

    import paper_2511_21713_amd as pb
    ctx = pb.Context(0)
    cases = [("rna20k", cached_config(1)), ("bumpy_n3", pbgen.make_problem(n=3, a=6.0, c=9.0, bump=True, t=3.0, L=3,
                                                                           helix=3, partials=5, kappa=0.2,
                                                                           seed=(9, 1)))]
    for name, prob in cases:  # the second call is on a smaller problem
        for precision in (pb.FP64, pb.MIXED):
            log(f"[noalloc] {name}, precision {precision}")
            g = pb.Problem.from_inputs(ctx, prob, precision=precision)
            g.setup()
            rng = np.random.default_rng(7)
            for scheme in (oracle.T3, oracle.HS):
                phi = 0.5 * rng.standard_normal(g.n)
                ref = g.residual(scheme, phi)
                dphi = torch.tensor(phi, device="cuda:0")
                out = torch.full((g.n,), np.nan, dtype=torch.float64, device="cuda:0")
                g.residual_noalloc(scheme, dphi, out, stream=torch.cuda.current_stream())
                torch.cuda.synchronize()
                got = out.cpu().numpy()
                err = np.abs(got - ref).max() / np.abs(ref).max()
                log(f"  scheme {scheme}: max rel diff to pbfb_residual {err:.2e}")
                assert np.array_equal(got, ref)
            g.close()
        if name == "bumpy_n3":  # small enough for the oracle: the same bar as pbfb_residual
            o = oracle.Oracle.from_problem(prob)
            g = pb.Problem.from_inputs(ctx, prob)
            g.setup()
            phi = 0.5 * np.random.default_rng(8).standard_normal(g.n)
            out = torch.zeros(g.n, dtype=torch.float64, device="cuda:0")
            g.residual_noalloc(oracle.HS, torch.tensor(phi, device="cuda:0"), out)
            torch.cuda.synchronize()
            r = o.residual(oracle.HS, phi)
            assert np.abs(out.cpu().numpy() - r).max() < 1e-12 * np.abs(r).max()
            g.close()
    ctx.close()


def test_noalloc_residual_errors():
    import torch

    import paper_2511_21713_amd as pb
    ctx = pb.Context(0)
    prob = cached_config(0)
    g = pb.Problem.from_inputs(ctx, prob)
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda:0")
    y = torch.zeros(g.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pb.PbfbError) as e:  # not set up: the entry point does not set up
        g.residual_noalloc(oracle.HS, x, y)
    assert e.value.code == pb.ESTATE
    g.setup()
    xh = np.zeros(g.n)
    code = pb.lib().pbfb_residual_noalloc(g.h, oracle.HS, xh.ctypes.data, y.data_ptr(), None)
    assert code == pb.EINVAL  # host memory
    g.residual_noalloc(oracle.HS, x, y)
    g.close()
    big = pb.Problem(ctx)  # 40962 vertices per interface: beyond the fixed work array
    p2 = cached_config(2)
    big.set_mesh(p2.nodes, p2.tets, p2.tri_m, p2.tri_s)
    with pytest.raises(pb.PbfbError) as e:
        big.residual_noalloc(oracle.HS, torch.zeros(big.n, dtype=torch.float64, device="cuda:0"),
                             torch.zeros(big.n, dtype=torch.float64, device="cuda:0"))
    log(f"  too large: {pb.last_error()}")
    assert e.value.code == pb.EINVAL
    big.close()
    ctx.close()
