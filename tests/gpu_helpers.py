"""Shared helpers of the GPU tests: run the C ABI on numpy inputs."""
import numpy as np


def analyze_gpu(odp, events, stream=None):
    """Runs odp_analyze_trace on a numpy array of 64-byte records; returns (flags, report dict)."""
    import torch
    ev = np.ascontiguousarray(events)
    n = ev.shape[0]
    raw = ev.view(np.uint8).reshape(-1)
    d_ev = torch.from_numpy(raw.copy()).to("cuda") if n else torch.zeros(64, dtype=torch.uint8, device="cuda")
    d_flags = torch.full((max(n, 1),), 0xAA, dtype=torch.uint8, device="cuda")
    d_rep = torch.zeros(odp.REPORT_BYTES, dtype=torch.uint8, device="cuda")
    odp.analyze_trace(d_ev, d_flags, d_rep, stream=stream, n=n)
    torch.cuda.synchronize()
    return d_flags[:n].cpu().numpy(), odp.report_to_dict(d_rep.cpu().numpy())


def compare(flags_gpu, rep_gpu, flags_ref, rep_ref):
    bad = np.nonzero(flags_gpu != flags_ref)[0]
    assert bad.size == 0, "flags differ at %s: gpu %s oracle %s" % (
        bad[:10].tolist(), flags_gpu[bad[:10]].tolist(), flags_ref[bad[:10]].tolist())
    diff = {k: (rep_gpu[k], rep_ref[k]) for k in rep_ref if rep_gpu[k] != rep_ref[k]}
    assert not diff, diff
