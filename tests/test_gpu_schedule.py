"""The forked schedule (near field on the plan's side stream, concurrently
with the far chain: the task flow of Sec. 3.2 pipelined as in Sec. 3.3) and
the pipelined one (also the leaf level's M2L beside the M2M chain) launch
the same kernels on the same data as the serial order, so their results are
bit-identical to it, in every precision mode, for repeated and back-to-back
evaluations on one stream."""
import numpy as np
import pytest
import torch

from paper_1206_0115_amd import fmm, inputs

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("sched", ["forked", "pipelined"])
@pytest.mark.parametrize("mode", ["fp64", "mixed", "fp64_svd", "mixed_svd"])
def test_concurrent_schedules_equal_serial(mode, sched):
    print(f"schedule parity {mode} {sched}", flush=True)
    pos, q = inputs.uniform_cube(60000, 77)
    # height 5: the leaf level's tiles and two coarser levels' tiles
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), 5, 5, mode)
    qd = torch.from_numpy(q).cuda()
    plan.set_schedule("serial")
    ref = [host(t) for t in plan.evaluate(qd)]
    plan.set_schedule(sched)
    # several evaluations queued back to back before any synchronisation
    outs = [plan.evaluate(qd) for _ in range(3)]
    torch.cuda.synchronize()
    for phi, f in outs:
        assert np.array_equal(host(phi), ref[0])
        assert np.array_equal(host(f), ref[1])
    plan.set_schedule("serial")
    parts_s = [host(t) for t in plan.evaluate_parts(qd)]
    plan.set_schedule(sched)
    parts_f = [host(t) for t in plan.evaluate_parts(qd)]
    for a, b in zip(parts_s, parts_f):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("split", [1, 3])
def test_pipelined_with_split_m2l_and_height_three(split):
    """The split compressed M2L (parts into partial buffers) and a tree whose
    only M2L level is the leaf level (no coarse launch) also agree bitwise."""
    for n, h in ((40000, 5), (3000, 3)):
        pos, q = inputs.sphere_surface(n, 79)
        plan = fmm.Plan(torch.from_numpy(pos).cuda(), h, 6, "mixed_svd")
        plan.set_m2l_split(split)
        qd = torch.from_numpy(q).cuda()
        plan.set_schedule("serial")
        ref = [host(t) for t in plan.evaluate(qd)]
        plan.set_schedule("pipelined")
        phi, f = plan.evaluate(qd)
        torch.cuda.synchronize()
        assert np.array_equal(host(phi), ref[0]) and np.array_equal(host(f), ref[1])


def test_forked_on_a_side_stream_and_bad_schedule():
    pos, q = inputs.sphere_surface(30000, 78)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = fmm.Plan(torch.from_numpy(pos).cuda(), 5, 4, stream=s)
        qd = torch.from_numpy(q).cuda()
        plan.set_schedule("serial")
        ref = [host(t) for t in plan.evaluate(qd, stream=s)]
        plan.set_schedule("forked")
        phi, f = plan.evaluate(qd, stream=s)
        s.synchronize()
    assert np.array_equal(host(phi), ref[0]) and np.array_equal(host(f), ref[1])
    with pytest.raises(fmm.FMMError):
        plan.set_schedule(7)


@pytest.mark.parametrize("sched", ["forked", "pipelined"])
def test_graph_replay_matches_eager(sched):
    """Evaluations replayed from the plan's captured hipGraph equal the eager
    launches bit for bit: several replays with different charges and output
    buffers, eager GPU work and synchronisations in between, and a new
    capture after the mode changes."""
    pos, q = inputs.uniform_cube(50000, 80)
    q2 = np.random.default_rng(81).uniform(-1.0, 1.0, len(q))
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), 5, 5)
    plan.set_schedule(sched)
    qs = [torch.from_numpy(q).cuda(), torch.from_numpy(q2).cuda()]
    for mode in ("fp64", "mixed_svd"):
        print(f"graph replay {sched} {mode}", flush=True)
        plan.set_precision(mode)
        plan.set_graph(False)
        ref = [[host(t) for t in plan.evaluate(qq)] for qq in qs]
        plan.set_graph(True)
        for k in range(5):
            phi, f = plan.evaluate(qs[k % 2])
            torch.cuda.synchronize()
            assert np.array_equal(host(phi), ref[k % 2][0]), (mode, k)
            assert np.array_equal(host(f), ref[k % 2][1]), (mode, k)
            x = torch.randn(512, 512, device="cuda")  # eager work between replays
            (x @ x).sum().item()
    plan.set_graph(False)
    phi, f = plan.evaluate(qs[0])
    assert np.array_equal(host(phi), ref[0][0]) and np.array_equal(host(f), ref[0][1])
    assert fmm.lib().fmm_plan_set_graph(plan.handle, 2) == fmm.FMM_ERR_ARG
