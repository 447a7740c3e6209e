"""Serving (continuous batching): requests arriving while others are on the
GPU are admitted into free column slots at their group's iteration
boundaries, groups of different mesh sizes run concurrently at their own
pace, and every result equals the same
request solved alone (bit for bit up to 1e-12 relative: a column's
arithmetic does not depend on its neighbours) and the oracle's direct
solve (1e-5 for the FP32-multigrid path, 1e-6 for FP64)."""

import numpy as np
import pytest
import torch

from oracle import solver as osolver
import workloads as W
from gpu_util import to_host, rel_l2

pytestmark = pytest.mark.gpu


def _rhs(req, M):
    f = np.stack([W.gaussian_nodal(2, req["n"], c, req["sigma"]) for c in req["centres"]])
    return np.stack([M @ fi for fi in f]).astype(np.complex128)


@pytest.mark.parametrize("precision,tol_err,sizes,count,max_cols", [
    ("fp32", 1e-5, (32, 64), 10, 4), ("fp64", 1e-6, (32, 64), 10, 4),
    # the register-streaming kernels on the finest levels; max_cols 3 makes
    # the server open a second group of a size when the first is full
    ("fp32", 1e-5, (128, 256), 8, 3)])
def test_serving_mix_matches_alone_and_oracle(precision, tol_err, sizes, count, max_cols):
    from paper_2506_18694_amd import Server, Solver
    reqs = W.serving_stream(count, sizes=sizes, max_rhs=3, seed=4)
    probs = {n: osolver.Problem(2, n, n / 10.0, n / 10.0, levels=int(np.log2(n / 8)) + 1)
             for n in sizes}
    srv = Server(hbm_budget_bytes=16e9, max_cols=max_cols, precision=precision)
    ids, xs, bs = {}, {}, {}
    pending = list(reqs)
    steps = 0
    while pending or any(srv.query(i)["status"] != 2 for i in ids.values()):
        # two arrivals every third step: later requests join running groups
        if pending and steps % 3 == 0:
            for req in pending[:2]:
                b = _rhs(req, probs[req["n"]].M)
                rid, x = srv.submit(torch.from_numpy(b).cuda(), req["n"], req["levels"], req["k"])
                ids[req["id"]], xs[req["id"]], bs[req["id"]] = rid, x, b
            pending = pending[2:]
        srv.step()
        steps += 1
        assert steps < 5000
    for req in reqs:
        info = srv.query(ids[req["id"]])
        assert info["status"] == 2 and info["converged"] == 1
        assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        x_mix = to_host(xs[req["id"]])
        s = Solver(2, req["n"], req["levels"], req["k"], 0.0, req["k"], precision=precision)
        x_alone, st = s.solve(torch.from_numpy(bs[req["id"]]).cuda(), tol=1e-8)
        s.close()
        assert rel_l2(x_mix, to_host(x_alone)) < 1e-12
        assert st["outer_its"] == info["outer_its"]
        pr = probs[req["n"]]
        for c in range(req["nrhs"]):
            u = pr.solve_direct(bs[req["id"]][c])
            assert rel_l2(x_mix[c], u) < tol_err
    srv.close()


def test_serving_budget_releases_idle_groups():
    """A budget that holds one group at a time: groups are released when
    idle and requests of the other size wait, then complete."""
    from paper_2506_18694_amd import Server, Solver
    reqs = W.serving_stream(6, sizes=(32, 64), max_rhs=2, seed=7)
    probe = Solver(2, 64, 4, 6.4, 0.0, 6.4, precision="fp32")
    one_group = probe.workspace_bytes(2) * 1.2
    probe.close()
    srv = Server(hbm_budget_bytes=one_group, max_cols=2, precision="fp32")
    probs = {n: osolver.Problem(2, n, n / 10.0, n / 10.0, levels=int(np.log2(n / 8)) + 1)
             for n in (32, 64)}
    out = []
    for req in reqs:
        b = _rhs(req, probs[req["n"]].M)
        rid, x = srv.submit(torch.from_numpy(b).cuda(), req["n"], req["levels"], req["k"])
        out.append((req, rid, x, b))
    steps = 0
    while any(srv.query(rid)["status"] != 2 for _, rid, _, _ in out):
        srv.step()
        q, r, used = srv.load()
        assert used <= one_group
        steps += 1
        assert steps < 5000
    for req, rid, x, b in out:
        assert srv.query(rid)["converged"] == 1
        xh = to_host(x)
        for c in range(req["nrhs"]):
            assert rel_l2(xh[c], probs[req["n"]].solve_direct(b[c])) < 1e-5
    srv.close()
