"""The serving loop through the C-ABI: every request's results are
bit-identical to the same evaluation run alone through fmm_evaluate, whatever
it is batched with (different N, order, height, precision, distribution);
admission under a small memory budget queues requests instead of failing;
a request larger than the budget is rejected with FMM_ERR_OOM."""
import numpy as np
import pytest
import torch

from paper_1206_0115_amd import fmm, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def make_requests(k, seed=0):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(k):
        n = int(np.exp(rng.uniform(np.log(2000), np.log(60000))))
        kind = "cube" if rng.random() < 0.5 else "sphere"
        l = int(rng.choice([3, 5, 7]))
        h = int(rng.integers(2, 6))
        prec = ["fp64", "mixed", "fp64_svd", "mixed_svd"][int(rng.integers(0, 4))]
        pos, q = inputs.make(kind, n, 500 + i)
        reqs.append((torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(), h, l, prec))
    return reqs


def alone(req):
    pos, q, h, l, prec = req
    p = fmm.Plan(pos, h, l, prec)
    phi, f = p.evaluate(q)
    torch.cuda.synchronize()
    out = phi.cpu().numpy(), f.cpu().numpy()
    p.release()
    return out


def test_results_identical_alone_and_in_the_mix():
    reqs = make_requests(14)
    ref = [alone(r) for r in reqs]
    srv = fmm.Server(hbm_budget_bytes=64 << 30, max_active=16)
    tickets = [srv.submit(pos, q, h, l, prec) for pos, q, h, l, prec in reqs]
    for i, t in enumerate(tickets):
        st = t.wait()
        assert st.status == fmm.FMM_OK, (i, st.status, fmm.last_error())
        assert np.array_equal(t.potential.cpu().numpy(), ref[i][0]), i
        assert np.array_equal(t.forces.cpu().numpy(), ref[i][1]), i
    s = srv.stats()
    say(f"batches {s.batches} max jobs {s.max_batch_jobs} captures {s.graph_captures}")
    assert s.completed == len(reqs) and s.rejected == 0
    assert s.max_batch_jobs >= 2  # requests really shared launches
    srv.close()


def leaf_height(pos, target=64.0):
    """Height whose non-empty leaves hold closest to `target` particles (the
    serving workload's rule), from the root cube of the positions."""
    lo = pos.min(axis=0)
    L = float((pos.max(axis=0) - lo).max()) or 1.0
    best, best_d = 2, None
    for h in range(2, 9):
        side = 2 ** (h - 1)
        k = np.minimum(np.floor((pos - lo) / L * side), side - 1).astype(np.int64)
        occ = len(pos) / len(np.unique((k[:, 0] * side + k[:, 1]) * side + k[:, 2]))
        d = abs(np.log(occ) - np.log(target))
        if best_d is None or d < best_d:
            best, best_d = h, d
    return best


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_serving_workload_mix_matches_oracle_and_solo_runs():
    """Requests shaped like the serving workload (N log-uniform in [1e4, 2e6]
    with one above 1e6, orders 3, 5, 7 and 9, cube or sphere, about 64
    particles per leaf): every served result equals its solo run bit for bit;
    FP64 results match the oracle at sampled targets within 1e-12, the mixed
    modes match the FP64 run within the 1e-6 gate, the compressed FP64 mode
    within 10 x its tolerance."""
    import oracle

    rng = np.random.default_rng(2024)
    orders = [9, 7, 5, 3, 9, 7, 5, 3]
    precs = ["fp64", "mixed_svd", "fp64_svd", "mixed", "mixed_svd", "fp64", "mixed", "fp64_svd"]
    reqs = []
    for i, (l, prec) in enumerate(zip(orders, precs)):
        n = 1_200_000 if i == 1 else int(np.exp(rng.uniform(np.log(1e4), np.log(2e6))))
        kind = "cube" if i % 2 == 0 else "sphere"
        pos, q = inputs.make(kind, n, 700 + i)
        h = leaf_height(pos)
        say(f"request {i}: {kind} n={n} h={h} l={l} {prec}")
        reqs.append((pos, q, h, l, prec))
    assert max(r[0].shape[0] for r in reqs) >= 1_000_000
    assert max(r[2] for r in reqs) >= 6
    dev = [(torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda(), h, l, prec)
           for p, q, h, l, prec in reqs]
    solo = [alone(r) for r in dev]
    srv = fmm.Server(hbm_budget_bytes=96 << 30, max_active=16)
    tickets = [srv.submit(pos, q, h, l, prec) for pos, q, h, l, prec in dev]
    out = []
    for i, t in enumerate(tickets):
        st = t.wait()
        assert st.status == fmm.FMM_OK, (i, st.status, fmm.last_error())
        phi, f = t.potential.cpu().numpy(), t.forces.cpu().numpy()
        assert np.array_equal(phi, solo[i][0]) and np.array_equal(f, solo[i][1]), i
        out.append((phi, f))
    s = srv.stats()
    say(f"batches {s.batches} max jobs {s.max_batch_jobs}")
    srv.close()
    for i, (pos, q, h, l, prec) in enumerate(reqs):
        phi, f = out[i]
        if prec == "fp64":
            idx = np.sort(np.random.default_rng(i).choice(len(q), 48, replace=False))
            p_o, f_o = oracle.Tree(pos, h).fmm(l, q, targets=idx)
            e = max(rel(phi[idx], p_o), rel(f[idx], f_o))
            say(f"  request {i} ({prec}, l={l}) vs oracle {e:.2e}")
            assert e <= 1e-12, (i, e)
        else:
            p64, f64 = alone(dev[i][:4] + ("fp64",))
            e = max(rel(phi, p64), rel(f, f64))
            say(f"  request {i} ({prec}, l={l}) vs fp64 {e:.2e}")
            bound = 1e-6 if prec.startswith("mixed") else 10 * 10.0 ** -min(l, 10)
            assert e <= bound, (i, e)


def test_arrivals_while_running_join_later_batches():
    reqs = make_requests(10, seed=3)
    ref = [alone(r) for r in reqs]
    srv = fmm.Server(hbm_budget_bytes=64 << 30, max_active=4)
    tickets = []
    for r in reqs:
        tickets.append(srv.submit(*r[:4], precision=r[4]))
    sts = [t.wait() for t in tickets]
    for i, t in enumerate(tickets):
        assert sts[i].status == fmm.FMM_OK
        assert np.array_equal(t.potential.cpu().numpy(), ref[i][0])
        assert np.array_equal(t.forces.cpu().numpy(), ref[i][1])
    s = srv.stats()
    assert s.max_active_seen <= 4 and s.batches >= 3
    srv.close()


def test_small_budget_queues_and_oversize_is_rejected():
    reqs = make_requests(6, seed=5)
    srv = fmm.Server(hbm_budget_bytes=1 << 30, max_active=8)
    first = [srv.submit(*r[:4], precision=r[4]) for r in reqs]
    sts = [t.wait() for t in first]
    foot = max(st.plan_bytes for st in sts)
    srv.close()
    # a budget that holds about two plans: everything still completes
    srv = fmm.Server(hbm_budget_bytes=int(2.2 * foot), max_active=8)
    tickets = [srv.submit(*r[:4], precision=r[4]) for r in reqs]
    for t in tickets:
        assert t.wait().status == fmm.FMM_OK
    s = srv.stats()
    assert s.peak_admitted_bytes <= int(2.2 * foot)
    # a request larger than the whole budget ends with FMM_ERR_OOM
    pos, q = inputs.uniform_cube(2_000_000, 9)
    big = srv.submit(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(), 7, 7)
    small = srv.submit(*reqs[0][:4], precision=reqs[0][4])
    assert big.wait().status == fmm.FMM_ERR_OOM
    assert small.wait().status == fmm.FMM_OK
    srv.close()


def test_submit_rejects_bad_arguments():
    srv = fmm.Server(hbm_budget_bytes=1 << 30, max_active=2)
    pos = torch.zeros(10, 3, dtype=torch.float64, device="cuda")
    q = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(fmm.FMMError):
        srv.submit(pos, q, 0, 5)
    with pytest.raises(fmm.FMMError):
        srv.submit(pos, q, 3, 13)
    srv.close()


def test_request_arriving_mid_batch_runs_beside_it():
    """A small request submitted while a large batch runs is planned at once
    and launched on the second table buffer's stream without waiting for the
    large batch; both results equal their solo runs bit for bit."""
    big_pos, big_q = inputs.uniform_cube(1_500_000, 71)
    small_pos, small_q = inputs.sphere_surface(20_000, 72)
    big = (torch.from_numpy(big_pos).cuda(), torch.from_numpy(big_q).cuda(), 6, 9, "fp64")
    small = (torch.from_numpy(small_pos).cuda(), torch.from_numpy(small_q).cuda(), 4, 3,
             "mixed")
    ref_big, ref_small = alone(big), alone(small)
    srv = fmm.Server(hbm_budget_bytes=64 << 30, max_active=8)
    srv.submit(*small[:4], precision=small[4]).wait()  # graphs and operators warm
    tb = srv.submit(*big[:4], precision=big[4])
    while True:  # the large batch has been launched
        st = tb.poll()
        if st is not None or srv.stats().batches >= 2:
            break
    ts = srv.submit(*small[:4], precision=small[4])
    sb, ss = tb.wait(), ts.wait()
    say(f"big: admit {sb.admit_s:.4f} done {sb.done_s:.4f} batch {sb.batch}; "
        f"small: submit {ss.submit_s:.4f} done {ss.done_s:.4f} batch {ss.batch}")
    assert sb.status == fmm.FMM_OK and ss.status == fmm.FMM_OK
    assert ss.batch != sb.batch and ss.submit_s < sb.done_s
    assert np.array_equal(tb.potential.cpu().numpy(), ref_big[0])
    assert np.array_equal(tb.forces.cpu().numpy(), ref_big[1])
    assert np.array_equal(ts.potential.cpu().numpy(), ref_small[0])
    assert np.array_equal(ts.forces.cpu().numpy(), ref_small[1])
    assert tb.error() == "" and ts.error() == ""
    srv.close()


def test_failed_plan_keeps_its_status_and_message():
    """A request whose positions are not finite ends with the plan's own
    status (FMM_ERR_ARG) and message; the server keeps serving."""
    pos, q = inputs.uniform_cube(5000, 73)
    pos[7, 2] = np.nan
    srv = fmm.Server(hbm_budget_bytes=8 << 30, max_active=4)
    bad = srv.submit(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(), 4, 4)
    st = bad.wait()
    assert st.status == fmm.FMM_ERR_ARG and "NaN" in bad.error()
    pos[7, 2] = 0.5
    good = srv.submit(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(), 4, 4)
    assert good.wait().status == fmm.FMM_OK and good.error() == ""
    srv.close()
