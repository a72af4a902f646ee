"""Stream and graph behaviour of the library: every call is queued on the caller's
stream with its own workspace, so independent calls on two streams may overlap; and
the whole fit step (forward, misfit, adjoint) can be captured in a HIP graph, since no
entry point allocates, synchronises or issues a memset.  Each graph replay is checked
bitwise against the eager result, with eager work and synchronisations between replays."""
import numpy as np
import pytest
import torch

from paper_1010_2641_amd import api, workloads as wl

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def problem(seed, n=3000, k=5000):
    xyz, f, S = wl.random_problem(n, k, seed=seed, extent=30.0, s_range=2.0)
    I = np.abs(wl.random_seed_field(k, seed=seed + 1, scale=40.0)).astype(np.float32) ** 2
    return dev(xyz), dev(f), dev(S), dev(I)


def test_two_streams_overlap_correctly():
    a = problem(111)
    b = problem(112, n=4100, k=3300)
    ref_a = [t.clone() for t in api.fit_step(*a)]
    ref_b = [t.clone() for t in api.fit_step(*b)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()        # default priority
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            oa = api.fit_step(*a)
        with torch.cuda.stream(s2):
            ob = api.fit_step(*b)
        outs.append((oa, ob))
    torch.cuda.synchronize()
    for oa, ob in outs:
        for x, y in zip(oa, ref_a):
            assert torch.equal(x, y)
        for x, y in zip(ob, ref_b):
            assert torch.equal(x, y)


def test_fit_step_in_a_graph():
    xs, fs, Ss, Is = problem(113)
    L0, A0, g0 = [t.clone() for t in api.fit_step(xs, fs, Ss, Is)]
    other = problem(114, n=500, k=700)
    # warm up on a side stream, then capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        api.fit_step(xs, fs, Ss, Is)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        L, A, g = api.fit_step(xs, fs, Ss, Is)
    for rep in range(4):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(L, L0) and torch.equal(A, A0) and torch.equal(g, g0), rep
        # eager work of the program between replays
        api.fit_step(*other)
        (A0.abs() ** 2).sum().item()
        torch.cuda.synchronize()
    # the graph reads its input buffers at replay time: new positions, new result
    xs2 = xs + 0.01
    L1, A1, g1 = [t.clone() for t in api.fit_step(xs2, fs, Ss, Is)]
    xs.copy_(xs2)
    for rep in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(L, L1) and torch.equal(A, A1) and torch.equal(g, g1), rep
