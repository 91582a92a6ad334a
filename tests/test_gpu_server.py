"""The request server: continuous batching and the FIFO loop give every request the image it
gets when solved alone with the same call sequence (bit for bit); the data-driven gamma
matches the oracle's; admission under a small memory budget queues instead of failing."""
from __future__ import annotations

import time

import numpy as np
import pytest

from gpu_common import say
from oracle import pd, problem
from paper_1801_02417_amd import psara as P
from paper_1801_02417_amd import workloads as wk

pytestmark = pytest.mark.gpu

STAGES = (8, 6, 6)
NORM_ITERS, NORM_RTOL = 60, 1e-7


def requests():
    out = []
    for i, (n, M, L) in enumerate([(16, 150, 2), (32, 600, 3), (64, 2500, 4), (32, 900, 2), (16, 300, 2),
                                   (64, 1200, 3)]):
        wl = wk.tiny(n=n, M=M, taps=8, levels=L, seed=100 + i)
        b = problem.build(wl, norm_rtol=1e-6, norm_max_iter=40)
        out.append((wl, b.pb.Y, b.pb.eps))
    return out


def solve_alone(wl, Y, eps, prec):
    ctx = P.psara_create(0)
    try:
        P.psara_set_operator(ctx, wl.n, wl.uv, 2, wl.taps, prec)
        P.psara_set_data(ctx, Y, eps)
        P.psara_set_prior(ctx, P.ALL_BASES, wl.levels, None, 1.0)
        P.psara_opnorm(ctx, NORM_ITERS, NORM_RTOL)
        P.psara_set_gamma(ctx, P.psara_data_gamma(ctx, 1e-3))
        P.psara_set_steps_auto(ctx, 0.99)
        P.psara_reweighted_solve(ctx, P.PSARA_CONSTRAINED, STAGES, 10.0)
        return P.psara_get_image(ctx, wl.n * wl.n)
    finally:
        P.psara_destroy(ctx)


def serve(reqs, prec, policy, budget=8 << 30, quantum=5):
    srv = P.psara_server_create(0, budget, 16, quantum, policy)
    try:
        tickets = [P.psara_server_submit(srv, wl.n, wl.uv, Y, eps, taps=wl.taps, levels=wl.levels, precision=prec,
                                         iters_per_stage=STAGES, opnorm_iters=NORM_ITERS, opnorm_rtol=NORM_RTOL)
                   for wl, Y, eps in reqs]
        P.psara_server_drain(srv)
        out = []
        for (wl, _, _), t in zip(reqs, tickets):
            img = np.empty((wl.n * wl.n, 4))
            r = P.psara_server_poll(srv, t, img)
            assert r["state"] == P.PSARA_REQ_DONE, (r, P.lib().psara_server_last_error(srv))
            assert r["report"]["iterations"] == sum(STAGES)
            assert r["t_submit"] <= r["t_start"] <= r["t_done"]
            out.append(img)
        with pytest.raises(P.PsaraError):
            P.psara_server_poll(srv, tickets[0])      # collected requests are forgotten
        return out
    finally:
        P.psara_server_destroy(srv)


@pytest.mark.parametrize("prec", [P.PSARA_FP32_MIXED, P.PSARA_FP64])
def test_served_equals_alone(prec):
    reqs = requests()
    alone = [solve_alone(wl, Y, eps, prec) for wl, Y, eps in reqs]
    for policy in (P.PSARA_SERVE_BATCHED, P.PSARA_SERVE_FIFO):
        t0 = time.time()
        served = serve(reqs, prec, policy)
        say(f"policy {policy} prec {prec}: {len(reqs)} requests in {time.time() - t0:.2f} s")
        for (wl, _, _), a, b in zip(reqs, alone, served):
            assert np.array_equal(a, b), f"{wl.name}: served image differs ({np.max(np.abs(a - b))})"


def test_small_budget_queues():
    reqs = requests()[:3]
    foot = max(P.psara_footprint(wl.n, wl.M, wl.taps, wl.levels) for wl, _, _ in reqs)
    served = serve(reqs, P.PSARA_FP32_MIXED, P.PSARA_SERVE_BATCHED, budget=foot + 1)
    alone = [solve_alone(wl, Y, eps, P.PSARA_FP32_MIXED) for wl, Y, eps in reqs]
    for a, b in zip(alone, served):
        assert np.array_equal(a, b)


def test_data_gamma_matches_oracle():
    wl = wk.blobs32()
    b = problem.build(wl)
    ctx = P.psara_create(0)
    try:
        P.psara_set_operator(ctx, wl.n, wl.uv, 2, wl.taps, P.PSARA_FP64)
        P.psara_set_data(ctx, b.pb.Y, b.pb.eps)
        P.psara_set_prior(ctx, P.ALL_BASES, wl.levels, None, 1.0)
        P.psara_opnorm(ctx, 1000, 1e-13)
        g = P.psara_data_gamma(ctx, 1e-3)
        say(f"gamma gpu {g:.15e} oracle {b.gamma:.15e}")
        assert abs(g - b.gamma) <= 1e-9 * b.gamma
    finally:
        P.psara_destroy(ctx)


def test_served_fp64_request_matches_oracle():
    """One served FP64 request (the 32x32 blob workload, Algorithm 2 with 100 + 100 + 100
    iterations) against the oracle's Algorithm 2 on the same data: the server computes its own
    ||phi||^2 (power iteration to 1e-13) and data-driven gamma, the oracle its own (to 1e-12), so
    the two runs share the step sizes and gamma to about 1e-12."""
    wl = wk.blobs32()
    b = problem.build(wl)
    stages = pd.split_iterations(wl.iters, wl.cycles + 1)
    ref, _, _ = pd.alg2(b.pb, b.gamma, stages, len(stages) - 1)
    srv = P.psara_server_create(0, 8 << 30, 4, 25)
    try:
        t = P.psara_server_submit(srv, wl.n, wl.uv, b.pb.Y, b.pb.eps, taps=wl.taps, levels=wl.levels,
                                  precision=P.PSARA_FP64, iters_per_stage=stages, opnorm_iters=2000,
                                  opnorm_rtol=1e-13)
        P.psara_server_drain(srv)
        img = np.empty((wl.n * wl.n, 4))
        r = P.psara_server_poll(srv, t, img)
        assert r["state"] == P.PSARA_REQ_DONE, (r, P.lib().psara_server_last_error(srv))
    finally:
        P.psara_server_destroy(srv)
    errs = [float(np.linalg.norm(img[:, i] - ref.S[:, i]) / np.linalg.norm(ref.S[:, i])) for i in range(4)]
    say(f"served FP64 request vs oracle: per-Stokes rel err {['%.2e' % e for e in errs]}; "
        f"iterations {r['report']['iterations']}")
    assert r["report"]["iterations"] == sum(stages)
    assert max(errs) <= 1e-9


def test_cancel_frees_the_slot():
    """One slot: a long request runs, a second waits; cancelling the running one ends it at the
    next round and the second is admitted and completes; a queued request cancels at once."""
    srv = P.psara_server_create(0, 8 << 30, 1, 5)
    try:
        reqs = requests()
        (wa, ya, ea), (wb, yb, eb), (wc, yc, ec) = reqs[2], reqs[0], reqs[1]
        ta = P.psara_server_submit(srv, wa.n, wa.uv, ya, ea, taps=wa.taps, levels=wa.levels,
                                   iters_per_stage=(200000, 10, 10), opnorm_iters=NORM_ITERS, opnorm_rtol=NORM_RTOL)
        for _ in range(20000):
            if P.psara_server_poll(srv, ta)["state"] == P.PSARA_REQ_RUNNING:
                break
            time.sleep(0.001)
        tb = P.psara_server_submit(srv, wb.n, wb.uv, yb, eb, taps=wb.taps, levels=wb.levels,
                                   iters_per_stage=STAGES, opnorm_iters=NORM_ITERS, opnorm_rtol=NORM_RTOL)
        tc = P.psara_server_submit(srv, wc.n, wc.uv, yc, ec, taps=wc.taps, levels=wc.levels,
                                   iters_per_stage=STAGES, opnorm_iters=NORM_ITERS, opnorm_rtol=NORM_RTOL)
        P.psara_server_cancel(srv, tc)
        assert P.psara_server_poll(srv, tc)["state"] == P.PSARA_REQ_CANCELLED
        assert P.psara_server_poll(srv, tb)["state"] == P.PSARA_REQ_QUEUED
        time.sleep(0.2)
        P.psara_server_cancel(srv, ta)
        P.psara_server_drain(srv)
        assert P.psara_server_poll(srv, ta)["state"] == P.PSARA_REQ_CANCELLED
        img = np.empty((wb.n * wb.n, 4))
        r = P.psara_server_poll(srv, tb, img)
        assert r["state"] == P.PSARA_REQ_DONE and r["report"]["iterations"] == sum(STAGES)
        assert np.array_equal(img, solve_alone(wb, yb, eb, P.PSARA_FP32_MIXED))
        with pytest.raises(P.PsaraError):
            P.psara_server_cancel(srv, tb)         # collected: unknown ticket
    finally:
        P.psara_server_destroy(srv)


def test_request_larger_than_the_device_is_refused():
    """A request whose footprint exceeds the device's memory is refused with PSARA_ENOMEM at
    submission (before its arrays are read: they hold 16 rows of the 2^31 - 1 declared)."""
    import ctypes as C
    srv = P.psara_server_create(0, 8 << 30, 4, 5)
    try:
        M = (1 << 31) - 1
        assert P.psara_footprint(1024, M, 8, 4, P.ALL_BASES, P.PSARA_FP64) > 300 << 30
        uv = np.zeros((16, 2))
        y = np.zeros((16, 8))
        stages = (C.c_int * 3)(10, 10, 10)
        req = P.PsaraRequest(1024, M, P._dptr(uv), P._dptr(y), 1.0, 8, 4, P.ALL_BASES, P.PSARA_FP64,
                             P.PSARA_CONSTRAINED, 2, stages, 10.0, 1e-3, 10, 1e-3, 0, P.PsaraStop(0.0, 0.0, 0.0))
        ticket = C.c_uint64()
        st = P.lib().psara_server_submit(srv, C.byref(req), C.byref(ticket))
        assert st == P.PSARA_ENOMEM, st
        assert b"device memory" in P.lib().psara_server_last_error(srv)
    finally:
        P.psara_server_destroy(srv)


def test_bad_request_rejected():
    srv = P.psara_server_create(0, 1 << 30, 4, 5)
    try:
        wl = wk.tiny(n=16, M=150, taps=8, levels=2, seed=1)
        with pytest.raises(P.PsaraError) as e:
            P.psara_server_submit(srv, wl.n, wl.uv, np.zeros((wl.M, 4), complex), -1.0)
        assert e.value.status == P.PSARA_EINVAL
        # a request that fails during set-up (taps 5) is reported failed, not hung
        t = P.psara_server_submit(srv, wl.n, wl.uv, np.ones((wl.M, 4), complex), 1.0, taps=5)
        P.psara_server_drain(srv)
        r = P.psara_server_poll(srv, t)
        assert r["state"] == P.PSARA_REQ_FAILED and r["status"] == P.PSARA_EINVAL
    finally:
        P.psara_server_destroy(srv)


ADAPT_BOUND, ADAPT_CHECK, ADAPT_STOP = 120, 10, (5e-3, 5e-4, 0.5)


def solve_alone_adaptive(wl, Y, eps, prec):
    ctx = P.psara_create(0)
    try:
        P.psara_set_operator(ctx, wl.n, wl.uv, 2, wl.taps, prec)
        P.psara_set_data(ctx, Y, eps)
        P.psara_set_prior(ctx, P.ALL_BASES, wl.levels, None, 1.0)
        P.psara_opnorm(ctx, NORM_ITERS, NORM_RTOL)
        P.psara_set_gamma(ctx, P.psara_data_gamma(ctx, 1e-3))
        P.psara_set_steps_auto(ctx, 0.99)
        its, rep = P.psara_reweighted_solve_adaptive(ctx, P.PSARA_CONSTRAINED, 2, ADAPT_BOUND, ADAPT_CHECK,
                                                     ADAPT_STOP, 10.0)
        return P.psara_get_image(ctx, wl.n * wl.n), rep["iterations"]
    finally:
        P.psara_destroy(ctx)


@pytest.mark.parametrize("policy", [P.PSARA_SERVE_BATCHED, P.PSARA_SERVE_FIFO])
def test_served_adaptive_equals_alone(policy):
    """Requests whose stages end by the stopping test leave the batch on their own; each gets
    bit for bit the image (and iteration count) of psara_reweighted_solve_adaptive alone, and
    at least one stops before its bounds."""
    reqs = requests()
    alone = [solve_alone_adaptive(wl, Y, eps, P.PSARA_FP32_MIXED) for wl, Y, eps in reqs]
    say(f"adaptive iterations alone: {[a[1] for a in alone]} (bound {3 * ADAPT_BOUND})")
    assert any(a[1] < 3 * ADAPT_BOUND for a in alone)
    srv = P.psara_server_create(0, 8 << 30, 16, 30, policy)
    try:
        tickets = [P.psara_server_submit(srv, wl.n, wl.uv, Y, eps, taps=wl.taps, levels=wl.levels,
                                         iters_per_stage=(ADAPT_BOUND,) * 3, opnorm_iters=NORM_ITERS,
                                         opnorm_rtol=NORM_RTOL, check_every=ADAPT_CHECK, stop=ADAPT_STOP)
                   for wl, Y, eps in reqs]
        P.psara_server_drain(srv)
        for (wl, _, _), t, (img_a, it_a) in zip(reqs, tickets, alone):
            img = np.empty((wl.n * wl.n, 4))
            r = P.psara_server_poll(srv, t, img)
            assert r["state"] == P.PSARA_REQ_DONE, (r, P.lib().psara_server_last_error(srv))
            assert r["report"]["iterations"] == it_a, (wl.name, r["report"]["iterations"], it_a)
            assert np.array_equal(img, img_a), f"{wl.name}: served image differs"
    finally:
        P.psara_server_destroy(srv)


def test_adaptive_request_validation():
    srv = P.psara_server_create(0, 8 << 30, 4, 8, P.PSARA_SERVE_BATCHED)
    try:
        wl, Y, eps = requests()[0]
        with pytest.raises(P.PsaraError):       # bounds must be multiples of check_every
            P.psara_server_submit(srv, wl.n, wl.uv, Y, eps, iters_per_stage=(15, 20, 20), check_every=10)
        with pytest.raises(P.PsaraError):
            P.psara_server_submit(srv, wl.n, wl.uv, Y, eps, iters_per_stage=(10, 20, 20), check_every=10,
                                  stop=(-1.0, 1e-3, 0.5))
    finally:
        P.psara_server_destroy(srv)
