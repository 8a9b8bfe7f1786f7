"""The batched digest that allocates nothing (odp_digest_buffers_noalloc):
through the C ABI, its digests equal odp_digest_buffers' on two calls in a
row, the second smaller than the first (the fixed array keeps the first
call's contents); sizes beyond its limits are refused (buffer count on the
host, level-1 nodes on the device)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make_buffers(rng, sizes):
    return [torch.from_numpy(rng.integers(0, 256, size=s, dtype=np.uint8)).to("cuda") for s in sizes]


def tables(bufs, offsets):
    ptrs = torch.tensor(np.array([b.data_ptr() + o for b, o in zip(bufs, offsets)], dtype=np.uint64).view(np.int64),
                        device="cuda")
    sizes = torch.tensor(np.array([b.numel() - o for b, o in zip(bufs, offsets)], dtype=np.uint64).view(np.int64),
                         device="cuda")
    return ptrs, sizes


def both_forms(odp, ptrs, sizes):
    n = sizes.numel()
    out_ref = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    out_na = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    odp.digest_buffers(ptrs, sizes, out_ref)
    odp.digest_buffers_noalloc(ptrs, sizes, out_na)
    torch.cuda.synchronize()
    assert odp.device_status() == odp.ODP_OK
    return out_ref.cpu().numpy().view(np.uint64), out_na.cpu().numpy().view(np.uint64)


def test_two_calls_second_smaller(odp):
    rng = np.random.default_rng(71)
    # first call: 3,000 buffers, every size class (empty, sub-leaf, one node,
    # multi-node up to a three-level tree), some at unaligned starts
    sizes1 = np.concatenate([
        rng.integers(0, 4097, size=2000), rng.integers(4097, 262145, size=900),
        rng.integers(262145, 3 << 20, size=96), [0, 4096, 17 * 262144 + 5, (64 << 20) + 4097]]).astype(np.int64)
    rng.shuffle(sizes1)
    offs1 = [int(rng.integers(0, 16)) if s > 16 and rng.random() < 0.3 else 0 for s in sizes1]
    bufs1 = make_buffers(rng, [int(s) + o for s, o in zip(sizes1, offs1)])
    p1, s1 = tables(bufs1, offs1)
    ref1, na1 = both_forms(odp, p1, s1)
    assert (na1 == ref1).all()
    host = [b.cpu().numpy()[o:] for b, o in zip(bufs1, offs1)]
    assert (na1 == oracle.d64_many(host)).all()
    # second call: fewer and smaller buffers, in the same array
    sizes2 = rng.integers(0, 300_000, size=37)
    bufs2 = make_buffers(rng, [int(s) for s in sizes2])
    p2, s2 = tables(bufs2, [0] * len(bufs2))
    ref2, na2 = both_forms(odp, p2, s2)
    assert (na2 == ref2).all()
    assert (na2 == oracle.d64_many([b.cpu().numpy() for b in bufs2])).all()


def test_buffer_count_above_limit_refused(odp):
    n = odp.NOALLOC_MAX_BUFFERS + 1
    ptrs = torch.zeros(n, dtype=torch.int64, device="cuda")
    sizes = torch.zeros(n, dtype=torch.int64, device="cuda")
    out = torch.zeros(n, dtype=torch.int64, device="cuda")
    rc = odp.load().odp_digest_buffers_noalloc(odp._ptr(ptrs), odp._ptr(sizes), n, odp._ptr(out), odp._stream(None))
    assert rc == odp.ODP_ERANGE
    assert b"maximum" in odp.load().odp_last_error_string()


def test_nodes_above_limit_found_on_device(odp):
    """64 views of one 256 MiB buffer (buffers may alias) hold 65,536 level-1
    nodes, the limit; a 65th view of 4,097 bytes adds one node more: every
    digest of that call is 0 and the device status reports ODP_ECAPACITY.
    The next call, exactly at the limit, is correct again."""
    big = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    big.random_(0, 256)
    n = 65
    ptrs = torch.full((n,), big.data_ptr(), dtype=torch.int64, device="cuda")
    sizes = torch.full((n,), big.numel(), dtype=torch.int64, device="cuda")
    sizes[64] = 4097
    out = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    odp.digest_buffers_noalloc(ptrs, sizes, out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 0).all()
    assert odp.device_status() == odp.ODP_ECAPACITY
    assert odp.device_status() == odp.ODP_OK  # reading clears it
    m = 64
    out2 = torch.full((m,), -1, dtype=torch.int64, device="cuda")
    odp.digest_buffers_noalloc(ptrs[:m], sizes[:m], out2)
    ref = torch.full((m,), -1, dtype=torch.int64, device="cuda")
    odp.digest_buffers(ptrs[:m], sizes[:m], ref)
    torch.cuda.synchronize()
    assert odp.device_status() == odp.ODP_OK
    got = out2.cpu().numpy()
    assert (got == ref.cpu().numpy()).all() and (got == got[0]).all() and got[0] != 0
