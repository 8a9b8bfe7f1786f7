"""GPU parity of the digest path (batched and per-buffer forms) against the
CPU oracle, bit-exact, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2601_12713_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev_bytes(arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda")


def both_forms(odp, tensors):
    b = odp.digest_tensors(tensors)
    p = odp.digest_tensors(tensors, plain=True)
    return b, p


SIZES = [0, 1, 7, 8, 31, 32, 33, 63, 64, 100, 255, 256, 257, 4095, 4096, 4097, 4100, 8191, 8192, 8193,
         65536, 262143, 262144, 262145, 300000, 64 * 262144, 64 * 262144 + 1, 4097 * 4096 + 3]


def test_sizes_every_class(odp):
    rng = np.random.default_rng(11)
    host = [rng.integers(0, 256, size=s, dtype=np.uint8) for s in SIZES]
    want = [oracle.d64(h) for h in host]
    t = [dev_bytes(h) for h in host]
    b, p = both_forms(odp, t)
    assert b.tolist() == want
    assert p.tolist() == want


def test_unaligned_starts(odp):
    rng = np.random.default_rng(12)
    base = dev_bytes(rng.integers(0, 256, size=600_000, dtype=np.uint8))
    host = base.cpu().numpy()
    views, want = [], []
    for off in list(range(16)) + [24, 40, 4096 + 3]:
        for size in [0, 5, 40, 4096, 5000, 300_000]:
            views.append(base[off:off + size])
            want.append(oracle.d64(host[off:off + size]))
    b, p = both_forms(odp, views)
    assert b.tolist() == want
    assert p.tolist() == want


def test_one_leaf_buffers_at_aligned_offsets(odp):
    # Buffers of at most one leaf at 16-byte aligned starts take the per-buffer
    # path that loads the whole leaf at once and reads its remainder from LDS:
    # every remainder class of the 32-byte stripe and of the 16-byte loads,
    # and lengths around the 1 KiB load boundaries.
    rng = np.random.default_rng(18)
    base = dev_bytes(rng.integers(0, 256, size=3 * 4096 + 64, dtype=np.uint8))
    host = base.cpu().numpy()
    sizes = list(range(0, 70)) + [95, 96, 97, 127, 128, 129, 1008, 1023, 1024, 1025, 1040, 2047, 2048, 2049,
                                  3071, 3072, 3073, 4063, 4064, 4065, 4080, 4095, 4096]
    views, want = [], []
    for off in [0, 16, 48, 4096 + 32]:
        for size in sizes:
            views.append(base[off:off + size])
            want.append(oracle.d64(host[off:off + size]))
    assert odp.digest_tensors(views, plain=True).tolist() == want
    assert odp.digest_tensors(views).tolist() == want


def test_same_bytes_same_digest_any_alignment(odp):
    rng = np.random.default_rng(13)
    src = rng.integers(0, 256, size=270_000, dtype=np.uint8)
    arena = torch.zeros(16 * 300_000, dtype=torch.uint8, device="cuda")
    views = []
    for k in range(16):
        o = k * 300_000 + k
        arena[o:o + src.size] = dev_bytes(src)
        views.append(arena[o:o + src.size])
    b, p = both_forms(odp, views)
    assert len(set(b.tolist())) == 1 and b[0] == oracle.d64(src) and (p == b).all()


def test_four_level_tree(odp):
    # 2^30 + 4097 bytes: 262146 leaves -> 4097 level-1 -> 65 -> 2 -> root at level 4.
    # Its first 2^30 bytes: 4096 level-1 -> 64 -> root at level 3, the largest
    # buffer whose upper levels the per-buffer form finishes under one ticket.
    n = (1 << 30) + 4097
    g = torch.Generator(device="cuda")
    g.manual_seed(14)
    t = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)
    host = t.cpu().numpy()
    want = [oracle.d64(host), oracle.d64(host[:1 << 30])]
    b, p = both_forms(odp, [t, t[:1 << 30]])
    assert b.tolist() == want and p.tolist() == want


def test_mixed_batch_random_sizes(odp):
    rng = np.random.default_rng(15)
    sizes = np.floor(np.exp(rng.uniform(0, np.log(3 << 20), size=3000))).astype(np.int64)
    sizes[rng.random(sizes.size) < 0.05] = 0
    host = [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in sizes]
    want = oracle.d64_many(host)
    t = [dev_bytes(h) for h in host]
    b, p = both_forms(odp, t)
    assert (b == want).all()
    assert (p == want).all()


def test_repeated_calls_graph_and_direct(odp):
    """Tickets reset themselves: repeated calls (graph replay and direct
    launches, several launch widths) give the same digests."""
    rng = np.random.default_rng(16)
    host = [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in [5_000_000, 17_000_000, 3000, 262144 * 65]]
    want = oracle.d64_many(host).tolist()
    t = [dev_bytes(h) for h in host]
    saved = odp.get_tuning()
    try:
        for use_graph in (1, 0, 1):
            for bpc in (1, 3, 8):
                odp.set_tuning(blocks_per_cu=bpc, use_graph=use_graph)
                for _ in range(3):
                    assert odp.digest_tensors(t).tolist() == want
    finally:
        odp.set_tuning(**saved)
    assert odp.device_status() == 0


# Level-1 nodes at every side of the one-wavefront split: whole buffers of
# 2, 16 and 17 leaves, a last node of one leaf, a last node alone in its
# level-2 group (65 and 64*64 + 1 level-1 nodes), and a full 64-node buffer.
SPLIT_SIZES = [4097, 16 * 4096, 16 * 4096 + 1, 32 * 4096, 262144 + 4096, 262144 + 65536, 262144 + 65537,
               64 * 262144, 64 * 262144 + 100, 65 * 262144 + 4096 * 16, 4096 * 262144 + 7]


def test_tuning_points_same_digests(odp):
    """Nine launch configurations (workgroups per CU, graph or direct, split
    between one-wavefront and one-workgroup nodes, items claimed at once)
    give the oracle's digests."""
    rng = np.random.default_rng(18)
    host = [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in SPLIT_SIZES]
    host += [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in rng.integers(1, 300_000, size=300)]
    want = oracle.d64_many(host).tolist()
    t = [dev_bytes(h) for h in host]
    saved = odp.get_tuning()
    try:
        for bpc, graph, split, chunk in [(8, 1, 65536, 1), (1, 1, 0, 1), (2, 0, 4096, 2), (4, 1, 16384, 4),
                                         (8, 0, 32768, 8), (3, 1, 65536, 3), (1, 1, 0, 16), (4, 0, 0, 5),
                                         (2, 1, 32768, 16)]:
            odp.set_tuning(blocks_per_cu=bpc, use_graph=graph, split_bytes=split, chunk_nodes=chunk)
            for _ in range(2):
                assert odp.digest_tensors(t).tolist() == want, (bpc, graph, split, chunk)
        with pytest.raises(odp.OdpError):
            odp.set_tuning(split_bytes=100)
        with pytest.raises(odp.OdpError):
            odp.set_tuning(chunk_nodes=17)
    finally:
        odp.set_tuning(**saved)
    assert odp.digest_tensors(t, plain=True).tolist() == want
    assert odp.device_status() == 0


def test_non_default_stream(odp):
    rng = np.random.default_rng(17)
    host = [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in [100, 70_000, 2_000_000]]
    want = oracle.d64_many(host).tolist()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t = [dev_bytes(h) for h in host]
        got = odp.digest_tensors(t, stream=s)
        gotp = odp.digest_tensors(t, stream=s, plain=True)
    assert got.tolist() == want and gotp.tolist() == want


def test_invalid_arguments(odp):
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(odp.OdpError) as e:
        odp.digest_buffers_plain([0], [16], out)
    assert e.value.code == odp.ODP_EINVAL
    # n = 0 is a no-op
    odp.digest_buffers_plain([], [], out)


def test_plain_small_workload_digests(odp):
    ps = W.PlainSmall(seed=1)
    want = [oracle.d64(s) for s in ps.snapshots]
    t = [dev_bytes(s) for s in ps.snapshots]
    b, p = both_forms(odp, t)
    assert p.tolist() == want and b.tolist() == want


def test_large_arrays_full_size(odp):
    """16 fp64 arrays of 2^25 elements, each sent 4 times: sampled digests
    against the oracle, and digest equality exactly where the bytes are equal."""
    la = W.LargeArrays(seed=2, device="cuda")
    la.materialize()
    got = odp.digest_tensors(la.snapshots, plain=True)
    gotb = odp.digest_tensors(la.snapshots)
    assert (got == gotb).all()
    for i in [0, 17, 40, 63]:
        assert int(got[i]) == oracle.d64(la.snapshots[i].cpu().numpy().view(np.uint8)), i
    for i in range(len(la.snapshots)):
        prev = [j for j in range(i) if la.array_of[j] == la.array_of[i]]
        if prev:
            assert (got[i] == got[prev[-1]]) == la.identical[i], i


def test_batched_digest_replayed_from_a_graph(odp):
    """The batched digest captured by the caller (plan and digest kernels, no
    memset nodes) replays correctly several times."""
    rng = np.random.default_rng(19)
    host = [rng.integers(0, 256, size=int(s), dtype=np.uint8) for s in [0, 100, 5000, 70_000, 262_145, 3_000_000]]
    want = oracle.d64_many(host).tolist()
    t = [dev_bytes(h) for h in host]
    n = len(t)
    dp = torch.tensor(np.array([x.data_ptr() for x in t], dtype=np.uint64).view(np.int64), device="cuda")
    ds = torch.tensor(np.array([x.numel() for x in t], dtype=np.uint64).view(np.int64), device="cuda")
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        odp.reserve(max_buffers=n, max_total_bytes=1 << 24, stream=s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        odp.digest_buffers(dp, ds, out, stream=s)
    for _ in range(3):
        out.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert out.cpu().numpy().view(np.uint64).tolist() == want
    assert odp.device_status() == 0


def test_batched_capacity_overflow_sets_status(odp):
    """A workspace reserved for 2,048 buffers and 1 MiB in all (room for
    2,052 level-1 nodes), then 100 views of one 16 MiB buffer (6,400 nodes)
    on the same stream: the plan does not fit, every digest of the call is 0
    and odp_device_status reports ODP_ECAPACITY once (then clears). The next
    call within the reserve is correct again."""
    s = torch.cuda.Stream()  # a fresh workspace
    rng = np.random.default_rng(41)
    host = [rng.integers(0, 256, size=16 << 20, dtype=np.uint8)] * 100
    t = [dev_bytes(host[0])] * 100
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        odp.reserve(max_buffers=2048, max_total_bytes=1 << 20, stream=s)
        got = odp.digest_tensors(t, stream=s)
    assert (got == 0).all()
    assert odp.device_status() == odp.ODP_ECAPACITY
    assert odp.device_status() == odp.ODP_OK
    with torch.cuda.stream(s):
        small = odp.digest_tensors(t[:1], stream=s)
    assert small.tolist() == [oracle.d64(host[0])]
    assert odp.device_status() == odp.ODP_OK
