"""GPU parity of one time step (predictor multi-corrector of Sec. 2.5 with the
reduced outlet models of Algorithm 1) against the CPU oracle: same corrector
count, residual histories, final state and outlet values, with the linear
systems solved tightly on both sides so the iterates agree to rounding of the
solves."""
import numpy as np
import pytest
import torch

from conftest import get_case
from oracle import discretization as dz
from oracle import krylov as kr
from oracle import newton as nt

pytestmark = pytest.mark.gpu

_CTX = {}


def ctx_for(name):
    from paper_1911_10814_amd import NsContext
    if name not in _CTX:
        _CTX[name] = NsContext(get_case(name)).bind()
    return _CTX[name]


def inputs(name, rcr, seed=3):
    c = get_case(name)
    N = c.n_nodes
    y_n = np.concatenate([c.v.ravel(), c.p])
    rng = np.random.default_rng(seed)
    ydot_n = rng.standard_normal(4 * N) * 0.5
    dm = np.concatenate([c.mask[:, :3].ravel(), c.mask[:, 3]]).astype(bool)
    ydot_n[dm] = 0.0
    a_raw, _, _ = dz.outlet_vectors(c)
    no = c.n_outlets
    Q_n = np.array([np.sum(a_raw[k] * c.v) for k in range(no)])
    if rcr == "meta":   # per-outlet Windkessel parameters of the workload, steady start
        w = c.meta["rcr"]
        Pi = w["Rd"] * Q_n
        model = nt.OutletModel(Rp=w["Rp"], C=w["C"], Rd=w["Rd"], Pd=np.zeros(no), Pi=Pi, P=w["Rp"] * Q_n + Pi,
                               Q=Q_n, n_ts=100)
    elif rcr:   # three-element Windkessel: R_p = R/10, R_d = 9R/10, C such that R_d C = 10 dt
        Rp, Rd = 0.1 * c.R, 0.9 * c.R
        C = 10 * c.dt / Rd
        Pi = Rd * Q_n
        model = nt.OutletModel(Rp=Rp, C=C, Rd=Rd, Pd=np.full(no, 2.0), Pi=Pi, P=Rp * Q_n + Pi + 2.0, Q=Q_n,
                               n_ts=50)
    else:
        model = nt.OutletModel(Rp=c.R.copy(), C=np.zeros(no), Rd=np.zeros(no), Pd=np.zeros(no), Pi=np.zeros(no),
                               P=c.R * Q_n, Q=Q_n)
    return c, y_n, ydot_n, model


@pytest.mark.parametrize("name,rcr", [("cube", False), ("channel2", False), ("channel2", True),
                                      ("pipe_tiny", False), ("plate_small", "meta"), ("unstr_channel", True)])
def test_time_step_matches_oracle(name, rcr):
    from paper_1911_10814_amd import SolveOptions
    c, y_n, ydot_n, model = inputs(name, rcr)
    nopt = dict(tol_R=1e-8, tol_A=1e-14, l_max=8)
    ctx = ctx_for(name)
    md = {"Rp": model.Rp, "C": model.C, "Rd": model.Rd, "Pd": model.Pd, "Pi": model.Pi, "P": model.P,
          "Q": model.Q, "n_ts": model.n_ts}
    y, ydot, info, out = ctx.time_step(y_n, ydot_n, rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, model=md,
                                       newton=nopt, opts=SolveOptions(rtol=1e-12, rtol_A=1e-10, rtol_S=1e-10,
                                                                      rtol_I=1e-10))
    print(name, rcr, {k: info[k] for k in ("iterations", "converged", "res0", "res", "lin_outer", "total_ms")},
          flush=True)
    yo, ydo, io, mo = nt.time_step(c, y_n, ydot_n, model, nt.NewtonOpts(**nopt),
                                   kr.SolveOpts(rtol=1e-12, rtol_A=1e-10, rtol_S=1e-10, rtol_I=1e-10))
    assert info["converged"] == 1 and io["converged"]
    assert info["iterations"] == io["iterations"]
    h, ho = np.array(info["res_hist"]), np.array(io["res_hist"])
    assert len(h) == len(ho)
    # residual norms agree while they are well above the solves' accuracy
    big = ho > 1e-6 * ho[0]
    assert np.allclose(h[big], ho[big], rtol=1e-8)
    yn, ydn = y.cpu().numpy(), ydot.cpu().numpy()
    assert np.linalg.norm(yn - yo) <= 1e-10 * np.linalg.norm(yo)
    assert np.linalg.norm(ydn - ydo) <= 1e-8 * np.linalg.norm(ydo)
    for k in ("Q", "P", "Pi"):
        assert np.allclose(out[k], getattr(mo, k), rtol=1e-9, atol=1e-12)


def test_time_step_fp32_inner_converges_to_the_same_state():
    from paper_1911_10814_amd import SolveOptions
    c, y_n, ydot_n, model = inputs("pipe_tiny", False)
    ctx = ctx_for("pipe_tiny")
    md = {"Rp": model.Rp, "P": model.P, "Q": model.Q}
    kw = dict(rho=c.rho, mu=c.mu, dt=c.dt, rho_inf=c.rho_inf, model=md, newton=dict(tol_R=1e-8, tol_A=1e-14))
    y64, _, i64, _ = ctx.time_step(y_n, ydot_n, opts=SolveOptions(), **kw)
    y32, _, i32, _ = ctx.time_step(y_n, ydot_n, opts=SolveOptions(precision="fp32_inner"), **kw)
    assert i64["converged"] == 1 and i32["converged"] == 1
    assert float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64)) <= 1e-8
