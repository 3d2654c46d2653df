"""linscan_knn_noalloc (the linear-scan kNN whose buffers sit in a fixed
device array of the library) against linscan_knn, through the C ABI,
element by element, ids and distances bit-exact: two calls in a row, the
second with a smaller input; a batch scanned in several slices; exact
re-runs of overflowed queries inside the array; the documented capacity
error; empty inputs."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import assert_same, as_u32, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def same_as_linscan(mih, dc, dq, k, what):
    ids, dists = mih.linscan_knn_noalloc(dc, dq, k)
    li, ld = mih.linscan_knn(dc, dq, k)
    assert_same(ids, dists, as_u32(li), as_u32(ld), what)
    return ids, dists


def test_noalloc_two_calls_second_smaller(mih):
    n1, nq1 = 300_007, 300
    codes1 = datagen.uniform_codes(n1, 64, 501)
    queries1 = datagen.uniform_codes(nq1, 64, 502)
    k1 = datagen.choice_u32(nq1, [1, 10, 100, 1000], 503)
    dc1, dq1 = to_dev(codes1), to_dev(queries1)
    print(f"noalloc call 1: n={n1} nq={nq1} bits=64 mixed k", flush=True)
    ids, dists = same_as_linscan(mih, dc1, dq1, k1.tolist(), "first call")
    oi, od = oracle.knn(codes1, queries1, k1)
    assert_same(ids, dists, oi, od, "first call vs oracle")
    n2, nq2 = 50_021, 17
    codes2 = datagen.uniform_codes(n2, 128, 504)
    queries2 = datagen.uniform_codes(nq2, 128, 505)
    print(f"noalloc call 2: n={n2} nq={nq2} bits=128 k=10", flush=True)
    ids, dists = same_as_linscan(mih, to_dev(codes2), to_dev(queries2), 10, "second, smaller call")
    oi, od = oracle.knn(codes2, queries2, 10)
    assert_same(ids, dists, oi, od, "second call vs oracle")


def test_noalloc_batch_in_several_slices(mih):
    # k = 1000 queries hold 16,000-entry buffers (~128 KB each): 2,500 of
    # them need three slices of the array's first half
    n, nq = 100_003, 2_500
    codes = datagen.uniform_codes(n, 64, 511)
    queries = datagen.uniform_codes(nq, 64, 512)
    print(f"noalloc slices: n={n} nq={nq} k=1000", flush=True)
    same_as_linscan(mih, to_dev(codes), to_dev(queries), 1000, "sliced batch")


def test_noalloc_rerun_inside_the_array(mih):
    # 9000 identical codes: the candidate buffer overflows and the query is
    # re-run with an exact capacity, carved from the same array
    base = datagen.uniform_codes(3, 128, 9)
    codes = np.concatenate([np.repeat(base[:1], 9000, axis=0), base[1:]], axis=0)
    queries = np.concatenate([base[:1], base[1:2] ^ np.uint64(5)], axis=0)
    dc, dq = to_dev(codes), to_dev(queries)
    for k in [1, 100, 4096]:
        print(f"noalloc rerun: ties k={k}", flush=True)
        ids, dists = same_as_linscan(mih, dc, dq, k, f"ties k={k}")
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"ties k={k} vs oracle")


def test_noalloc_capacity_error_when_a_rerun_cannot_fit(mih):
    # 36 M identical codes tie with the query: its exact re-run needs 36 M
    # entries (288 MB), more than the whole array holds
    import torch
    n = 36_000_000
    dc = torch.full((n, 1), 12345, dtype=torch.int64, device="cuda")
    dq = torch.full((1, 1), 12345, dtype=torch.int64, device="cuda")
    print(f"noalloc capacity: n={n} identical codes k=1", flush=True)
    with pytest.raises(mih.MihError) as ei:
        mih.linscan_knn_noalloc(dc, dq, 1)
    assert ei.value.status == 5
    li, ld = mih.linscan_knn(dc, dq, 1)
    assert int(li[0, 0]) == 0 and int(ld[0, 0]) == 0
    # the array is usable again afterwards
    codes = datagen.uniform_codes(10_000, 64, 521)
    queries = datagen.uniform_codes(5, 64, 522)
    same_as_linscan(mih, to_dev(codes), to_dev(queries), 7, "after the capacity error")


def test_noalloc_empty_inputs(mih):
    import torch
    codes = datagen.uniform_codes(100, 64, 1)
    q = datagen.uniform_codes(3, 64, 2)
    empty = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    ids, dists = mih.linscan_knn_noalloc(empty, to_dev(q), 5)
    assert (ids.cpu() == -1).all() and (dists.cpu() == -1).all()
    ids, dists = mih.linscan_knn_noalloc(to_dev(codes), empty, 5)
    assert ids.numel() == 0
    with pytest.raises(mih.MihError):
        mih.linscan_knn_noalloc(to_dev(codes), to_dev(codes[:1]), 5000)
