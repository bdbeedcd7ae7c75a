"""Serving on the GPU: every request's frames and threshold are the same when
served alone and in a mix of concurrent requests (bit-identical: the same
kernels on the same resident level), also when eviction forces volumes to be
loaded and reduced again; one served result is checked against the oracle."""
import numpy as np
import pytest
import torch

from oracle import reduce as O
from oracle import render as R
from paper_2311_15038_amd import serve as S
from paper_2311_15038_amd import synth

from gpu_util import banner, dev

pytestmark = pytest.mark.gpu

EDGES = np.array([24, 40, 57, 64, 80, 33, 96, 48])


@pytest.fixture(scope="module")
def store():
    ex = S.GpuExecutor(EDGES, slots=1, seed_base=9100)
    for v in range(len(EDGES)):
        ex.host_volume(v)
    torch.cuda.synchronize()
    return ex.store


def _mix(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        out.append((float(rng.uniform(0, 0.02)),
                    S.Request(k, int(rng.integers(0, len(EDGES))), int(rng.integers(1, 7)),
                              int(rng.choice([256, 512])))))
    return out


def _alone(store, r):
    ex = S.GpuExecutor(EDGES, slots=1, seed_base=9100, store=store)
    srv = S.Server(ex, 1 << 34, slots=1)
    q = srv.submit(S.Request(r.rid, r.vol_id, r.n_views, r.res))
    srv.drain()
    assert q.status == "done", q.error
    return q.result


def _check_against_alone(store, trace):
    for _, r in trace:
        assert r.status == "done", (r.rid, r.status, r.error)
        frames, res = r.result
        f1, res1 = _alone(store, r)
        assert torch.equal(res, res1), r.rid
        assert torch.equal(frames, f1), r.rid


def test_mix_equals_alone(store):
    banner("serve: mix of 24 requests on 4 slots vs alone")
    ex = S.GpuExecutor(EDGES, slots=4, seed_base=9100, store=store)
    srv = S.Server(ex, 1 << 34, slots=4)
    trace = _mix(1, 24)
    st = srv.run(trace)
    assert st.done == 24 and st.failed == 0
    assert st.loads == len({r.vol_id for _, r in trace}) and st.max_inflight > 1
    _check_against_alone(store, trace)


def test_mix_with_eviction_equals_alone(store):
    banner("serve: tight budget, evictions")
    ex = S.GpuExecutor(EDGES, slots=4, seed_base=9100, store=store)
    big = max(ex.volume_bytes(S.Request(0, v, 1, 256)) for v in range(len(EDGES)))
    budget = 2 * big + 6 * 512 * 512 * 16          # two volumes + the largest request's frames
    srv = S.Server(ex, budget, slots=4)
    trace = _mix(2, 20)
    st = srv.run(trace)
    assert st.done == 20 and st.evictions > 0 and st.peak_bytes <= budget
    assert len(ex.vols) == len(srv.resident)
    _check_against_alone(store, trace)


def test_served_result_matches_oracle(store):
    banner("serve: one request vs the oracle")
    vid = 1                                    # 40^3 volume, 20^3 level
    ex = S.GpuExecutor(EDGES, slots=2, seed_base=9100, store=store)
    srv = S.Server(ex, 1 << 34, slots=2)
    r = srv.submit(S.Request(0, vid, 2, 256))
    srv.drain()
    frames, res = r.result
    a = store[vid].numpy().view(np.uint16)
    H, Ht = O.histogram(a), O.histogram(a, 0, 3)
    T = O.valley_threshold(H)
    assert int(res[0].item()) == T
    L1 = O.pyramid(a, O.keep_bits(T, Ht), 1)[0]
    cams = synth.turntable_cameras(*L1.shape[::-1], n_views=2)
    ref, _ = R.render(L1, (1, 1, 1), synth.default_tf().astype(np.float64), cams, 256, 256, 0.5)
    assert np.abs(frames.cpu().numpy() - ref).max() <= 2e-4


def test_bad_request_does_not_stop_the_loop(store):
    banner("serve: invalid requests")
    ex = S.GpuExecutor(EDGES, slots=2, seed_base=9100, store=store)
    srv = S.Server(ex, 1 << 34, slots=2)
    rs = [S.Request(0, 99, 1, 256), S.Request(1, 0, 49, 256), S.Request(2, 0, 2, 300),
          S.Request(3, 0, 2, 256)]
    srv.run([(0.0, r) for r in rs])
    assert [r.status for r in rs] == ["failed", "failed", "failed", "done"]
    assert all("VR_ERR" in r.error for r in rs[:3])
