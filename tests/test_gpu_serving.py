"""The serving loop on the GPU: a mixed Poisson stream over two parameter
sets, continuous batching with overlap between the sets; every request's
result equals the result of that request served alone, and decrypts to the
plaintext fasttext scores."""

import numpy as np
import pytest

import synth as S
from oracle import ptmatvec as PM
from synth.configs import WorkloadConfig

pytestmark = pytest.mark.gpu


def test_mixed_stream_results_independent_of_batching():
    import torch
    assert torch.cuda.is_available()
    from paper_1908_06972_amd.inference import encrypted_inference
    from paper_1908_06972_amd.serving import GpuExecutor, Scheduler, build_sets, poisson_trace
    specs = {"n12": WorkloadConfig("n12", 12, 4, 60, 40, 2, 60, 2, 40),
             "n13": WorkloadConfig("n13", 13, 4, 60, 40, 2, 60, 2, 40)}
    H, O = S.bow_weights(7, 4096, 16, 4)
    sets, policies, words, counts = build_sets(specs, H, O, pool_size=6, level=4, draws=S)
    trace = poisson_trace(505, 40, 2000.0, {"n12": 2, "n13": 1}, {k: 6 for k in specs}, words)
    stats = Scheduler(GpuExecutor(sets), policies, budget_bytes=8 << 30).run(trace)
    s = stats.summary()
    assert s["completed"] == len(trace) and s["rejected"] == 0
    assert s["mean_batch"] > 1.0                       # requests were batched
    for r in trace:
        ctx, model, pool = sets[r.pset]
        alone = encrypted_inference(ctx, model, [pool[r.doc]], [r.words])[0]
        mixed = r.result
        assert np.array_equal(ctx.export(alone), ctx.export(mixed)), r.rid
        lp = ctx.params
        got = lp.decode(ctx.decrypt(mixed), mixed.scale, model.classes).real
        want = PM.inference_plain(counts[r.pset][r.doc].astype(np.float64), H, O, r.words)
        assert np.max(np.abs(got - want)) <= 1e-5
