"""GPU tests of the continuous-batching server (through the C ABI).

Results against the FP64 oracle; bitwise equality of a request's image alone
and in a mix (arrivals while others run, admission by footprint,
cancellation of a co-scheduled request)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_2078_amd import sl1m
from paper_1310_2078_amd import workloads as W

pytestmark = pytest.mark.gpu
GIB = 1 << 30


def say(*a):
    print(*a, flush=True)


def _req(seed, n_pix, n_vis, kind=W.PIX_DELTA, sigma=0.0, gains=False, n_src=4):
    wl = W.small_random(seed, n_pix, n_vis, half_extent=0.1, uv_radius=600.0, w_sigma=80.0,
                        kind=kind, sigma=sigma, with_gains=gains)
    rng = np.random.default_rng(seed + 1000)
    x = np.zeros(n_pix)
    x[rng.choice(n_pix, n_src, replace=False)] = rng.uniform(0.5, 2.0, n_src)
    op = O.Operator(O.Problem.from_workload(wl), dense=n_pix * n_vis <= 4_000_000)
    V = op.forward(x) + 0.01 * (rng.standard_normal(n_vis) + 1j * rng.standard_normal(n_vis))
    return wl, op, V


def test_server_matches_oracle_with_given_L():
    say("[case] server vs oracle, L given")
    cases = [_req(1, 700, 1500), _req(2, 900, 1100, kind=W.PIX_GAUSS_WIDE, sigma=3e-3),
             _req(3, 600, 1300, gains=True)]
    srv = sl1m.Server(2 * GIB, max_slots=8)
    tickets = []
    for wl, op, V in cases:
        L, _ = O.power_iteration(op, 30)
        tickets.append((srv.submit(wl, V, 0.05, 40, L=L), L))
    srv.drain([t for t, _ in tickets])
    for (wl, op, V), (t, L) in zip(cases, tickets):
        ok, info, _ = srv.poll(t)
        ref = O.fista(op, V, L, 0.05, 40)
        img = srv.result(t).cpu().numpy()
        err = np.max(np.abs(img - ref.image)) / np.max(ref.image)
        say(f"    n_pix={wl.n_pix} err/peak {err:.2e} F {info['F']:.6g} vs {ref.F:.6g}")
        assert ok and info["status"] == 0
        assert err <= 1e-4
        assert abs(info["F"] - ref.F) <= 1e-4 * ref.F
        assert info["nnz"] == ref.nnz


def test_server_power_iteration_L():
    say("[case] server power iteration")
    wl, op, V = _req(4, 800, 1200)
    _, rq = O.power_iteration(op, 30, seed=7)
    srv = sl1m.Server(1 * GIB, max_slots=4)
    t = srv.submit(wl, V, 0.05, 5, L=0.0, power_iters=30, seed=7)
    srv.drain([t])
    info = srv.poll(t)[1]
    say(f"    L {info['L']:.9g} vs 1.01*rq {1.01 * rq:.9g}")
    assert abs(info["L"] - 1.01 * rq) <= 1e-5 * rq


def _alone(wl, V, **kw):
    srv = sl1m.Server(2 * GIB, max_slots=4)
    t = srv.submit(wl, V, 0.05, 30, **kw)
    srv.drain([t])
    return srv.result(t).cpu().numpy().copy(), srv.poll(t)[1]


def test_alone_equals_in_mix_with_arrivals_and_cancel():
    """Request X alone vs X arriving while Y runs, with Z cancelled mid-run."""
    say("[case] alone == in mix")
    X = _req(5, 1500, 2500)
    Y = _req(6, 2500, 3000, kind=W.PIX_GAUSS_WIDE, sigma=2e-3)
    Z = _req(7, 1000, 1000)
    ax, ix = _alone(X[0], X[2], L=0.0)
    ay, iy = _alone(Y[0], Y[2], L=0.0)
    srv = sl1m.Server(2 * GIB, max_slots=8, round_budget=2e7)
    ty = srv.submit(Y[0], Y[2], 0.05, 30)
    srv.step()
    srv.step()
    tz = srv.submit(Z[0], Z[2], 0.05, 30)
    # plans are built by the server's admission thread: step until Z runs
    for _ in range(1_000_000):
        srv.step()
        if srv.poll(tz)[2][1] > 0:
            break
    else:
        raise AssertionError("request never admitted")
    tx = srv.submit(X[0], X[2], 0.05, 30)
    for _ in range(5):
        srv.step()
    # every active request takes part in every round, so Z's last round is the
    # last one launched before the cancel; Z may be reported done (its vis and
    # img_out free to reuse) only once that round has completed
    r_cancel = srv.stats()["rounds"]
    srv.cancel(tz)
    for _ in range(1_000_000):
        if srv.poll(tz)[0]:
            assert srv.stats()["completed_rounds"] >= r_cancel
            break
        srv.step()
    else:
        raise AssertionError("cancelled request never reported done")
    srv.drain([tx, ty, tz])
    assert np.array_equal(srv.result(tx).cpu().numpy(), ax)
    assert np.array_equal(srv.result(ty).cpu().numpy(), ay)
    assert srv.poll(tx)[1]["F"] == ix["F"] and srv.poll(ty)[1]["L"] == iy["L"]
    assert srv.poll(tz)[1]["status"] == sl1m.ECANCELLED
    st = srv.stats()
    assert st["active"] == 0 and st["pending"] == 0


def test_admission_by_footprint():
    """Two requests that do not fit the arena together: the second waits until
    the first has finished, and both equal their results alone."""
    say("[case] admission by footprint")
    wl = W.small_random(21, 8000, 6000, half_extent=0.1, uv_radius=600.0, w_sigma=80.0)
    rng = np.random.default_rng(0)
    V1 = 10 * (rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis))
    V2 = 10 * (rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis))
    probe = sl1m.Plan.from_workload(wl, tile_blocks=2048)
    fp = probe.workspace_bytes + 4 * wl.n_pix + 8 * (wl.n_vis // 256 + 2 * wl.n_pix // 256 + 8) + 4096
    probe.close()
    a1, _ = _alone(wl, V1, L=0.0)
    a2, _ = _alone(wl, V2, L=0.0)
    srv = sl1m.Server((2 << 20) + int(1.5 * fp), max_slots=8, round_budget=4e7)
    t1 = srv.submit(wl, V1, 0.05, 30)
    t2 = srv.submit(wl, V2, 0.05, 30)
    # the first is admitted once the admission thread has built its plan; the
    # second stays pending (not reserved) while the first holds the arena
    a, p = srv.step()
    for _ in range(1_000_000):
        if a >= 1:
            break
        a, p = srv.step()
    say(f"    footprint {fp} B; once the first runs active={a} pending={p}")
    assert a == 1 and p == 1 and not srv.poll(t2)[0] and srv.poll(t2)[2][1] == 0
    srv.drain([t1, t2])
    assert np.array_equal(srv.result(t1).cpu().numpy(), a1)
    assert np.array_equal(srv.result(t2).cpu().numpy(), a2)


def test_cancel_while_admitting_then_serve():
    """A request cancelled right after its first step, while the admission
    thread may still be building its plan: it ends cancelled with its memory
    and slot returned, and the server then serves the next request exactly
    as alone."""
    say("[case] cancel during admission")
    wl, _, V = _req(12, 6000, 8000)
    X = _req(13, 1200, 1500)
    ax, ix = _alone(X[0], X[2], L=0.0)
    srv = sl1m.Server(1 * GIB, max_slots=1)
    t = srv.submit(wl, V, 0.05, 30)
    srv.step()
    srv.cancel(t)
    for _ in range(1_000_000):
        if srv.poll(t)[0]:
            break
        srv.step()
    else:
        raise AssertionError("cancelled request never reported done")
    assert srv.poll(t)[1]["status"] == sl1m.ECANCELLED
    st = srv.stats()
    say(f"    after the cancel: {st}")
    assert st["active"] == 0 and st["pending"] == 0 and st["arena_used"] == 0
    tx = srv.submit(X[0], X[2], 0.05, 30)   # needs the only slot
    srv.drain([tx])
    assert np.array_equal(srv.result(tx).cpu().numpy(), ax)
    assert srv.poll(tx)[1]["F"] == ix["F"]


def test_server_close_to_standalone_solve():
    say("[case] server vs sl1m_solve")
    wl, op, V = _req(9, 1200, 2000)
    L, _ = O.power_iteration(op, 30)
    plan = sl1m.Plan.from_workload(wl)
    img_s, info_s = plan.solve(V, 0.05, 60, L=L)
    srv = sl1m.Server(1 * GIB, max_slots=2)
    t = srv.submit(wl, V, 0.05, 60, L=L)
    srv.drain([t])
    img = srv.result(t).cpu().numpy()
    a = img_s.cpu().numpy()
    err = np.max(np.abs(img - a)) / np.max(a)
    say(f"    err/peak {err:.2e}")
    assert err <= 1e-5


def _grid_req(seed, n_side, kind=W.PIX_DELTA, sigma=0.0, n_vis=2000, gains=False, n_src=4):
    """A request on a centred n_side^2 grid over +-0.1 (grid evaluation)."""
    wl = W.small_random(seed, 10, n_vis, half_extent=0.1, uv_radius=600.0, w_sigma=80.0,
                        with_gains=gains)
    l, m, _ = W.grid_pixels(n_side, 0.1)
    wl.l, wl.m = l, m
    wl.sigma = np.full(l.size, sigma)
    wl.kind = np.full(l.size, kind, np.uint8)
    rng = np.random.default_rng(seed + 1000)
    x = np.zeros(l.size)
    x[rng.choice(l.size, n_src, replace=False)] = rng.uniform(0.5, 2.0, n_src)
    op = O.Operator(O.Problem.from_workload(wl), dense=l.size * n_vis <= 4_000_000)
    V = op.forward(x) + 0.01 * (rng.standard_normal(n_vis) + 1j * rng.standard_normal(n_vis))
    return wl, op, V


def test_server_grid_requests_match_oracle():
    """Requests whose pixels form one grid segment run the batched grid
    kernels (prep, forward, adjoint); results against the oracle's FISTA."""
    say("[case] server grid requests vs oracle")
    cases = [_grid_req(31, 40), _grid_req(32, 36, kind=W.PIX_GAUSS_WIDE, sigma=2e-3, gains=True),
             _grid_req(33, 34, kind=W.PIX_GAUSS_PARAXIAL, sigma=1.5e-3)]
    for wl, _, _ in cases:
        assert sl1m.Plan.from_workload(wl, grid="require").info()["grid"] == 1
    srv = sl1m.Server(2 * GIB, max_slots=8)
    tickets = []
    for wl, op, V in cases:
        L, _ = O.power_iteration(op, 30)
        tickets.append((srv.submit(wl, V, 0.05, 40, L=L), L))
    srv.drain([t for t, _ in tickets])
    for (wl, op, V), (t, L) in zip(cases, tickets):
        ok, info, _ = srv.poll(t)
        ref = O.fista(op, V, L, 0.05, 40)
        img = srv.result(t).cpu().numpy()
        err = np.max(np.abs(img - ref.image)) / np.max(ref.image)
        say(f"    n_pix={wl.n_pix} kind={wl.kind[0]} err/peak {err:.2e} F {info['F']:.6g} vs {ref.F:.6g}")
        assert ok and info["status"] == 0
        assert err <= 1e-4
        assert abs(info["F"] - ref.F) <= 1e-4 * ref.F


@pytest.mark.parametrize("policy", ["fair", "oldest"])
def test_server_grid_alone_equals_in_mix(policy):
    """Grid delta, grid Gaussian and a direct (irregular) request in one mix,
    with power iteration and a cancellation, under either round policy: each
    image bitwise equal to the same request alone, and close to the
    standalone grid solve."""
    say(f"[case] server grid alone == in mix, policy {policy}")
    X = _grid_req(41, 48)
    Y = _grid_req(42, 40, kind=W.PIX_GAUSS_WIDE, sigma=2e-3)
    Z = _req(43, 1500, 1800)
    ax, ix = _alone(X[0], X[2], L=0.0)
    ay, iy = _alone(Y[0], Y[2], L=0.0)
    az, _ = _alone(Z[0], Z[2], L=0.0)
    srv = sl1m.Server(2 * GIB, max_slots=8, round_budget=2e7, policy=policy)
    tz = srv.submit(Z[0], Z[2], 0.05, 30)
    srv.step()
    ty = srv.submit(Y[0], Y[2], 0.05, 30)
    srv.step()
    tx = srv.submit(X[0], X[2], 0.05, 30)
    w = srv.submit(Z[0], Z[2], 0.05, 30)     # cancelled while it runs
    for _ in range(4):
        srv.step()
    srv.cancel(w)
    srv.drain([tx, ty, tz, w])
    assert np.array_equal(srv.result(tx).cpu().numpy(), ax)
    assert np.array_equal(srv.result(ty).cpu().numpy(), ay)
    assert np.array_equal(srv.result(tz).cpu().numpy(), az)
    assert srv.poll(tx)[1]["F"] == ix["F"] and srv.poll(ty)[1]["L"] == iy["L"]
    assert srv.poll(w)[1]["status"] == sl1m.ECANCELLED
    for (wl, _, V), img, info in ((X, ax, ix), (Y, ay, iy)):
        plan = sl1m.Plan.from_workload(wl, grid="require")
        ref, _ = plan.solve(V, 0.05, 30, L=info["L"])
        ref = ref.cpu().numpy()
        err = np.max(np.abs(img - ref)) / np.max(ref)
        say(f"    n_pix={wl.n_pix} server vs standalone grid solve err/peak {err:.2e}")
        assert err <= 1e-5


def test_served_request_at_config5_largest_size():
    """A request at the top of the serving stream's ranges: 262,144
    wide-field Gaussian pixels (sigma = 2 spacings) on the stream's truncated
    row-major grid over +-0.05 and 200,000 visibilities, 200 iterations.  The
    served image against the same solve through sl1m_solve on a plan in
    caller memory (same L), within 1e-5 of the peak; that plan's operators
    against the oracle on sampled outputs (norm-relative 1e-5 and the
    element-wise bound)."""
    import elementwise as E
    wl = W.config5_request(0, np_range=(262144, 262144), nv_range=(200_000, 200_000))
    wl.kind = np.full(wl.n_pix, W.PIX_GAUSS_WIDE, np.uint8)
    wl.sigma = np.full(wl.n_pix, 2.0 * wl.meta["delta"])
    say(f"[case] served request n_pix={wl.n_pix} n_vis={wl.n_vis} Gaussian, 200 iterations")
    plan = sl1m.Plan.from_workload(wl)
    say(f"    plan info {plan.info()}")
    p = O.Problem.from_workload(wl)
    rng = np.random.default_rng(77)
    x = rng.standard_normal(wl.n_pix)
    r = rng.standard_normal(wl.n_vis) + 1j * rng.standard_normal(wl.n_vis)
    ks = np.arange(0, wl.n_vis, 2003)
    js = np.arange(0, wl.n_pix, 2621)
    Vg = plan.forward(x).cpu().numpy()[ks]
    gg = plan.adjoint(r).cpu().numpy()[js]
    Vo, go = O.forward_rows(p, x, ks), O.adjoint_cols(p, r, js)
    ef = np.linalg.norm(Vg - Vo) / np.linalg.norm(Vo)
    ea = np.linalg.norm(gg - go) / np.linalg.norm(go)
    wf = E.worst_ratio(Vg, Vo, E.abs_forward_rows(p, x, ks), wl.n_pix)
    wa = E.worst_ratio(gg, go, E.abs_adjoint_cols(p, r, js), wl.n_vis)
    say(f"    plan vs oracle sampled forward {ef:.3e} adjoint {ea:.3e} "
        f"element-wise {wf:.3e} {wa:.3e}")
    assert ef <= 1e-5 and ea <= 1e-5 and wf <= 1.0 and wa <= 1.0
    V = plan.forward(wl.x_true) + torch.as_tensor(wl.noise, dtype=torch.complex64,
                                                  device=plan.device)
    L = 1.01 * plan.estimate_L(30, seed=0)
    img_s, info_s = plan.solve(V, wl.lam, wl.n_iter, L=L)
    img_s = img_s.cpu().numpy()
    plan.close()
    srv = sl1m.Server(8 * GIB, max_slots=4)
    t = srv.submit(wl, V, wl.lam, wl.n_iter, L=L)
    srv.drain([t])
    ok, info, _ = srv.poll(t)
    img = srv.result(t).cpu().numpy()
    err = float(np.max(np.abs(img - img_s))) / float(np.max(img_s))
    say(f"    served vs sl1m_solve err/peak {err:.2e}  F {info['F']:.9g} vs {info_s['F']:.9g}")
    assert ok and info["status"] == 0
    assert err <= 1e-5
    assert abs(info["F"] - info_s["F"]) <= 1e-5 * info_s["F"]
    srv.close()


def _burst_request(rng, i):
    """Request i of the burst: direct delta, direct Gaussian, grid delta or
    grid Gaussian pixels (i mod 4), sizes drawn from rng, random data."""
    n_vis = int(rng.integers(800, 2500))
    kind = W.PIX_DELTA if i % 2 == 0 else W.PIX_GAUSS_WIDE
    sigma = 0.0 if kind == W.PIX_DELTA else 2e-3
    if i % 4 < 2:
        wl = W.small_random(200 + i, int(rng.integers(800, 2500)), n_vis, half_extent=0.1,
                            uv_radius=600.0, w_sigma=80.0, kind=kind, sigma=sigma,
                            with_gains=i % 3 == 0)
    else:
        wl = W.small_random(200 + i, 10, n_vis, half_extent=0.1, uv_radius=600.0,
                            w_sigma=80.0, with_gains=i % 3 == 0)
        l, m, _ = W.grid_pixels(int(rng.integers(16, 28)) * 2, 0.1)
        wl.l, wl.m = l, m
        wl.sigma = np.full(l.size, sigma)
        wl.kind = np.full(l.size, kind, np.uint8)
    V = 10 * (rng.standard_normal(n_vis) + 1j * rng.standard_normal(n_vis))
    return wl, V


def test_burst_with_cancels_equals_alone():
    """24 requests of four kinds submitted in one burst to a server with 6
    slots (the plans built by its admission thread while rounds run), four of
    them cancelled in different states (waiting, just reserved, running, late
    in the run): every other request's image and objective equal the same
    request served alone, bitwise, and the server ends empty."""
    say("[case] burst of 24 with cancels")
    rng = np.random.default_rng(77)
    reqs = [_burst_request(rng, i) for i in range(24)]
    alone = [_alone(wl, V, L=0.0) for wl, V in reqs]
    srv = sl1m.Server(2 * GIB, max_slots=6, round_budget=2e7)
    tk = [srv.submit(wl, V, 0.05, 30) for wl, V in reqs]
    srv.cancel(tk[3])          # waiting: never reserved
    srv.step()
    srv.cancel(tk[5])          # reserved by that step, its plan maybe still being built
    cancelled = {3, 5}
    settled = set()   # 15 and 21 once cancelled or found finished first
    late = None
    for _ in range(1_000_000):
        srv.step()
        if 15 not in settled:
            done15, _, times15 = srv.poll(tk[15])
            if times15[1] > 0:      # running (no step between this poll and the cancel)
                if not done15:
                    srv.cancel(tk[15])
                    cancelled.add(15)
                settled.add(15)
        if 21 not in settled:
            done21, _, times21 = srv.poll(tk[21])
            if late is None and times21[1] > 0:
                late = srv.stats()["rounds"] + 3
            if done21:
                settled.add(21)
            elif late is not None and srv.stats()["rounds"] >= late:
                srv.cancel(tk[21])  # late in its run
                cancelled.add(21)
                settled.add(21)
        if all(srv.poll(t)[0] for t in tk):
            break
    else:
        raise AssertionError("burst never drained")
    say(f"    cancelled {sorted(cancelled)}")
    for i, t in enumerate(tk):
        done, info, _ = srv.poll(t)
        assert done
        if i in cancelled:
            assert info["status"] == sl1m.ECANCELLED
            continue
        assert info["status"] == 0
        assert np.array_equal(srv.result(t).cpu().numpy(), alone[i][0]), f"request {i}"
        assert info["F"] == alone[i][1]["F"], f"request {i}"
    st = srv.stats()
    assert st["active"] == 0 and st["pending"] == 0 and st["arena_used"] == 0
