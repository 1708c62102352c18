"""Serving session on the GPU: every request's result equals its oracle solve and its
solve alone, whatever else shares the device (continuous batching), and the session
admits by footprint, refuses what it cannot hold, and returns all memory."""
import numpy as np
import pytest

import oracle
from paper_2605_29604_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def T():
    from paper_2605_29604_amd import tcmis
    return tcmis


def mixed_requests(count, seed):
    spec = gen.batch_spec(count, seed=seed, n_min=100, n_max=20000)
    graphs = [gen.make(*s) for s in spec]
    graphs += [gen.grid(s, s, s, 0.01, seed + s) for s in (5, 12, 20)]
    graphs.insert(3, gen.er(0, 0, 1))      # empty request
    graphs.insert(5, gen.er(1, 0, 1))      # one vertex
    return graphs


def footprint(g, **opts):
    r = lambda x: (x + 255) // 256 * 256
    return (r(T().mis_build_bytes(g.n, g.nnz, **opts)) + r((g.n + 1) * 8) + r(g.nnz * 4) + r(max(g.n, 1)))


def pinned(a):
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


def drive(sess, graphs, opts_of=lambda i: None, step_poll=False):
    """Admits requests in order as the session accepts them; returns per-request
    (host result, done record), how often admission was refused, the most live.
    step_poll: drive the session with separate step and poll calls instead of progress."""
    pending = list(range(len(graphs)))
    outs, done = {}, {}
    busy = most_live = 0
    inputs = {i: (pinned(g.row_ptr), pinned(g.col_idx)) for i, g in enumerate(graphs)}
    while pending or sess.query()[0] > 0:
        while pending:
            i = pending[0]
            h = torch.zeros(max(graphs[i].n, 1), dtype=torch.uint8).pin_memory()
            if not sess.admit(*inputs[i], tag=i, host_out=h, opts=opts_of(i)):
                busy += 1
                break
            outs[i] = h
            pending.pop(0)
            print(f"admit request {i} n={graphs[i].n}", flush=True)
        most_live = max(most_live, sess.query()[0])
        if step_poll:
            sess.step()
            retired = sess.poll(wait=False)
        else:
            retired = sess.progress(wait=True)
        for d in retired:
            assert d["status"] == 0
            done[d["tag"]] = d
    return {i: (outs[i].numpy()[: graphs[i].n], done[i]) for i in outs}, busy, most_live


def alone(g, seed=1, **opts):
    t = T()
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    h = t.mis_build_tiles(rp, ci, seed=seed, **opts)
    out, st = t.mis_solve(h)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    t.mis_free_tiles(h)
    return res, st["rounds"]


def test_session_mix_equals_alone_and_oracle():
    graphs = mixed_requests(30, seed=21)
    biggest = max(footprint(g) for g in graphs)
    sess = T().Session(arena_bytes=(5 * biggest) // 2, max_live=6, rounds_per_step=2)
    res, busy, most_live = drive(sess, graphs)
    print(f"session: refused {busy} admissions, up to {most_live} live", flush=True)
    assert busy > 0 and most_live > 1
    for i, g in enumerate(graphs):
        got, d = res[i]
        st, rounds, _ = oracle.roundsync(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 1))
        want = (st == oracle.IN).astype(np.uint8)
        assert np.array_equal(got, want), f"request {i}"
        assert d["rounds"] == rounds and d["n_in"] == int(want.sum()) and d["n"] == g.n
        if i % 4 == 0 and g.n > 0:
            a, r = alone(g)
            assert np.array_equal(a, got) and r == d["rounds"], f"request {i} alone"
    live, used, largest = sess.query()
    assert live == 0 and used == 0 and largest == sess.arena.numel() // 256 * 256
    sess.close()


def test_session_step_and_poll_driven_separately():
    # the same continuous batching, driven by separate step (enqueue the next rounds)
    # and poll (retire) calls: every result equals the oracle's
    graphs = mixed_requests(16, seed=5)
    biggest = max(footprint(g) for g in graphs)
    sess = T().Session(arena_bytes=3 * biggest, max_live=4, rounds_per_step=1)
    res, busy, most_live = drive(sess, graphs, step_poll=True)
    print(f"session step/poll: refused {busy} admissions, up to {most_live} live", flush=True)
    assert most_live > 1
    for i, g in enumerate(graphs):
        got, d = res[i]
        st, rounds, _ = oracle.roundsync(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 1))
        assert np.array_equal(got, (st == oracle.IN).astype(np.uint8)), f"request {i}"
        assert d["rounds"] == rounds
    assert sess.step() == 0 and sess.poll(wait=True) == []
    sess.close()


def test_session_one_at_a_time_device_inputs_and_per_request_options():
    t = T()
    graphs = mixed_requests(10, seed=33)
    options = [dict(path="tile", tile=32, reorder="degree", seed=5), dict(path="csr", seed=5)]
    need = max(footprint(g, **{k: v for k, v in o.items() if k != "seed"}) for g in graphs for o in options)
    sess = t.Session(arena_bytes=2 * need, max_live=1, rounds_per_step=3)
    outs = {}
    for i, g in enumerate(graphs):
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx).cuda()
        out = torch.zeros(max(g.n, 1), dtype=torch.uint8, device="cuda")
        opts = options[i % 2]
        assert sess.admit(rp, ci, tag=100 + i, out=out, opts=opts)
        assert not sess.admit(rp, ci, tag=999, out=out)         # the one slot is taken
        (d,) = sess.progress(wait=True)
        assert d["tag"] == 100 + i
        torch.cuda.synchronize()
        outs[i] = out.cpu().numpy()[: g.n]
        st, rounds, _ = oracle.roundsync(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 5))
        assert np.array_equal(outs[i], (st == oracle.IN).astype(np.uint8)) and d["rounds"] == rounds
    sess.close()


def test_session_refuses_requests_larger_than_the_arena():
    t = T()
    small, big = gen.er(500, 2000, 1), gen.rmat(1 << 14, 8 << 14, 1)
    sess = t.Session(arena_bytes=footprint(small) + 4096, max_live=2)
    with pytest.raises(t.MisError) as ei:
        sess.admit(big.row_ptr, big.col_idx, tag=1, host_out=np.zeros(big.n, np.uint8))
    assert ei.value.code == t.MIS_EINVAL
    h = np.zeros(small.n, np.uint8)
    assert sess.admit(small.row_ptr, small.col_idx, tag=2, host_out=h)
    (d,) = sess.progress(wait=True)
    st, rounds, _ = oracle.roundsync(small.row_ptr, small.col_idx, oracle.keys(small.row_ptr, 1))
    assert np.array_equal(h, (st == oracle.IN).astype(np.uint8)) and d["rounds"] == rounds
    sess.close()


def test_session_refuses_persistent_launch():
    # concurrent requests each on their own stream cannot all hold a device-filling
    # cooperative grid, so the session refuses persistent launches before any work
    t = T()
    small = gen.er(500, 2000, 1)
    sess = t.Session(arena_bytes=4 * footprint(small), max_live=2)
    with pytest.raises(t.MisError) as ei:
        sess.admit(small.row_ptr, small.col_idx, tag=1, host_out=np.zeros(small.n, np.uint8),
                   opts=dict(launch="persistent"))
    assert ei.value.code == t.MIS_EINVAL
    assert sess.query()[0] == 0
    sess.close()
