"""Serving loop on the GPU: a seeded request mix served with continuous
batching on several streams gives every request the bit-identical result it
gets alone, and the results match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from conftest import fp64_err
from paper_2311_14670_amd.synth import serving_trace

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def test_mix_equals_alone_and_oracle():
    from paper_2311_14670_amd import binding, serving
    binding.load_library()
    trace = serving_trace(n_requests=48, seed=3, rate=1e4, lmin=8, lmax=96, so3_lmax=24)
    reqs = serving.build_requests(trace, seed=3)
    ex = serving.GpuExecutor(n_streams=3, max_batch=4)
    try:
        sched = serving.Scheduler(ex, hbm_budget=8 << 30)
        serving.serve(sched, reqs, realtime=False)
    finally:
        ex.close()
    assert not sched.rejected and len(sched.done) == len(reqs)
    assert max(r.batch_size for r in reqs) > 1           # some requests were really batched

    # alone: a fresh plan of batch 1 per request, default stream
    for r in reqs:
        k = r.key
        plan = binding.Plan(k.L, spin=k.spin, N=k.N, sampling=k.sampling, nside=k.nside)
        x = torch.from_numpy(r.data).cuda()
        if k.kind == "so3":
            y = plan.so3_forward(plan.so3_inverse(x))
        else:
            y = plan.forward(plan.inverse(x))
        alone = y.cpu().numpy()
        assert np.array_equal(alone, r.result), f"request {r.rid} {k} differs from its batch-{r.batch_size} result"
        plan.close()

    # oracle: exact round trips for MW / SO(3); HEALPix against the oracle's own pair
    for r in reqs[:16]:
        k = r.key
        if k.kind == "so3":
            ref = oracle.so3_forward(oracle.so3_inverse(r.data, k.L, k.N), k.L, k.N)
        elif k.sampling == "mw":
            ref = oracle.s2_forward(oracle.s2_inverse(r.data, k.L, k.spin), k.L, k.spin)
        else:
            f = oracle.s2_inverse(r.data, k.L, k.spin, oracle.HEALPIX, k.nside)
            ref = oracle.s2_forward(f, k.L, k.spin, oracle.HEALPIX, k.nside)
        assert fp64_err(r.result, ref) < 1e-12, (r.rid, k)


def test_mixed_precision_mix_matches_fp64():
    """The same mix served with the split-BF16 contraction: every result within the
    split-BF16 tolerance of the FP64 result, and equal to the request served alone
    with that precision (the matrix-core path does not depend on batch composition)."""
    from paper_2311_14670_amd import binding, serving
    binding.load_library()
    trace = serving_trace(n_requests=24, seed=5, rate=1e4, lmin=8, lmax=96, so3_lmax=24)
    for spec in trace:
        spec["precision"] = "split_bf16"
    reqs = serving.build_requests(trace, seed=5)
    ex = serving.GpuExecutor(n_streams=2, max_batch=4, min_mfma_batch=1)   # every batch on the matrix cores
    try:
        sched = serving.Scheduler(ex, hbm_budget=8 << 30)
        serving.serve(sched, reqs, realtime=False)
    finally:
        ex.close()
    assert not sched.rejected and len(sched.done) == len(reqs)
    assert all(r.run_precision == "split_bf16" for r in reqs)
    for r in reqs:
        k = r.key
        x = torch.from_numpy(r.data).cuda()
        outs = []
        for prec in ("split_bf16", "fp64"):
            plan = binding.Plan(k.L, spin=k.spin, N=k.N, sampling=k.sampling, nside=k.nside, precision=prec)
            y = plan.so3_forward(plan.so3_inverse(x)) if k.kind == "so3" else plan.forward(plan.inverse(x))
            outs.append(y.cpu().numpy())
            plan.close()
        assert np.array_equal(outs[0], r.result), (r.rid, k)
        assert rel_l2(r.result, outs[1]) < 2e-4, (r.rid, k)
        assert rel_l2(r.result, outs[1]) > 1e-12          # the reduced-precision products were used


def test_small_matrix_core_batches_run_fp64():
    """Default policy: a split-BF16 batch of fewer than four maps runs on the FP64
    plan (faster and more accurate there); a larger one on the matrix cores.  Each
    result equals the request served alone at the precision its batch ran with."""
    from paper_2311_14670_amd import binding, serving
    binding.load_library()
    specs = [dict(kind="s2", L=48, spin=0, sampling="mw", precision="split_bf16", t=0.0)] * 6
    specs += [dict(kind="s2", L=40, spin=2, sampling="mw", precision="split_bf16", t=0.0),
              dict(kind="so3", L=16, N=3, sampling="mw", precision="split_bf16", t=0.0)]
    reqs = serving.build_requests(specs, seed=7)
    ex = serving.GpuExecutor(n_streams=2, max_batch=8)
    try:
        sched = serving.Scheduler(ex, hbm_budget=8 << 30)
        serving.serve(sched, reqs, realtime=False)
    finally:
        ex.close()
    assert not sched.rejected and len(sched.done) == len(reqs)
    by = {r.rid: r for r in reqs}
    assert all(by[i].run_precision == "split_bf16" and by[i].batch_size == 6 for i in range(6))
    assert by[6].run_precision == "fp64" and by[7].run_precision == "fp64"
    for r in reqs:
        k = r.key
        plan = binding.Plan(k.L, spin=k.spin, N=k.N, sampling=k.sampling, nside=k.nside, precision=r.run_precision)
        x = torch.from_numpy(r.data).cuda()
        y = plan.so3_forward(plan.so3_inverse(x)) if k.kind == "so3" else plan.forward(plan.inverse(x))
        assert np.array_equal(y.cpu().numpy(), r.result), (r.rid, k, r.run_precision)
        plan.close()
