"""The serving loop: every request's result is bit-identical alone and in a
concurrent mix, matches the oracle, respects the HBM budget, and repeated
matrices hit the on-device stage-1 cache."""

import numpy as np
import pytest

from hlf_inputs import grid_instance, serve_requests
from oracle import c_oracle as C
from oracle import hlf_oracle as O
from paper_2103_00693_amd import hlf
from paper_2103_00693_amd.serve import Request, Server

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def make_requests(count=24, seed=0, n_max=32):
    reqs = serve_requests(count, rate_per_s=1000.0, master_seed=seed, n_min=4, n_max=n_max)
    out = [Request(rid=k, A=q["A"], seed=q["seed"], arrival=q["t"]) for k, q in enumerate(reqs)]
    # a repeated matrix (cache) and an invalid one (error path)
    out.append(Request(rid=len(out), A=out[0].A.copy(), seed=out[0].seed, arrival=out[-1].arrival))
    bad = grid_instance(6, seed=3)
    bad[0, 9] = 1
    out.append(Request(rid=len(out), A=bad, seed=5, arrival=out[-1].arrival))
    return out


def by_rid(results):
    return {r.rid: r for r in results}


def test_alone_equals_mix_and_oracle():
    reqs = make_requests()
    print("[serve] mix", flush=True)
    mix = by_rid(Server(slots=8, num_samples=4096).run(reqs, realtime=False))
    alone = {}
    for q in reqs:
        print(f"[serve] alone rid={q.rid} n={q.A.shape[0]}", flush=True)
        r = Server(slots=1, num_samples=4096, cache_entries=0).run([q], realtime=False)
        alone[q.rid] = r[0]
    assert set(mix) == set(alone) == {q.rid for q in reqs}
    for q in reqs:
        a, m = alone[q.rid], mix[q.rid]
        assert (a.status, a.rank, a.kind) == (m.status, m.rank, m.kind), q.rid
        if a.data is None:
            assert m.data is None
        else:
            assert np.array_equal(a.data, m.data), q.rid
    assert mix[reqs[-1].rid].status == hlf.HLF_ENOTSYM and mix[reqs[-1].rid].kind == "error"
    # oracle: enumerations exactly, samples: first rows exactly + kernel equations for all
    for q in reqs[:-1]:
        res = mix[q.rid]
        Fo = O.factor(q.A)
        assert res.rank == Fo["rank"]
        if res.kind == "enumerate":
            ref = C.enumerate_range(Fo, 0, 1 << Fo["rank"])[:, 0]
            got = res.data.view(np.uint16 if res.data.dtype == np.int16 else
                                np.uint32 if res.data.dtype == np.int32 else np.uint64).astype(np.uint64)
            assert np.array_equal(got, ref), q.rid
        else:
            Z = res.data.view(np.uint64).reshape(-1, Fo["words"])
            head = [sum(int(Z[s, w]) << (64 * w) for w in range(Fo["words"])) for s in range(8)]
            assert head == O.sample(Fo, q.seed, 8), q.rid
            free = [c for c in range(Fo["n"]) if c not in set(Fo["pivots"])]
            for f, kf in zip(free, Fo["kernel"]):
                kw = np.array([(kf >> (64 * w)) & ((1 << 64) - 1) for w in range(Fo["words"])],
                              dtype=np.uint64)
                par = np.bitwise_count(Z & kw).sum(axis=1) & 1
                assert np.all(par == ((Fo["shift"] >> f) & 1)), (q.rid, f)


def test_budget_cache_and_realtime():
    reqs = make_requests(count=30, seed=1)
    srv = Server(slots=4, num_samples=4096)
    budget = 3 * max(srv.footprint(q.A.shape[0]) for q in reqs)
    srv = Server(slots=4, num_samples=4096, hbm_budget=budget)
    print(f"[serve] realtime, budget={budget}", flush=True)
    res = by_rid(srv.run(reqs, realtime=True))
    assert len(res) == len(reqs)
    assert srv.max_in_flight <= budget
    dup = reqs[-2]
    assert res[dup.rid].cache_hit or res[0].cache_hit
    assert np.array_equal(res[dup.rid].data, res[0].data)
    assert all(r.latency > 0 for r in res.values())
