"""nomad_eval_rmse_noalloc (the evaluation for callers that cannot allocate device memory)
against nomad_eval_rmse on the same context: two calls in a row, the second on a smaller
input, in a fresh process or after the other tests.  Both are FP64 sums with Neumaier
compensation over different reduction trees, so they agree to well within 1e-12 relative."""
import numpy as np
import pytest
import torch

import paper_1312_0193_amd as nm
import synth

pytestmark = pytest.mark.gpu


def test_noalloc_evaluation_matches_the_allocating_one():
    prob = synth.small_case(3_000, 1_200, 150_000, seed=61, k=48, test_frac=0.2)
    hp = prob.hp
    W0, H0 = synth.init_factors(prob.m, prob.n, hp["k"], 61)
    print("[case] noalloc evaluation, k=48, 16 workers", flush=True)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp["k"], lam=hp["lam"],
                     alpha=hp["alpha"], beta=hp["beta"], gamma=hp["gamma"], workers=16, seed=3)
    model.train(2)
    dev = torch.device("cuda")
    tr, tc, tv = (x.to(dev).contiguous() for x in (prob.test_row, prob.test_col, prob.test_val))
    out = torch.full((3,), -1.0, dtype=torch.float64, device=dev)
    sizes = [tr.numel(), 7_777]  # the second call is smaller: nothing left over from the first
    assert sizes[0] > 2 * 8192 + 17  # the first spans several partial blocks and a ragged tail
    for nnz in sizes:
        r, j = model.evaluate(tr[:nnz], tc[:nnz], tv[:nnz])
        model.evaluate_noalloc(tr[:nnz], tc[:nnz], tv[:nnz], out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert got[2] == 0.0
        assert got[0] == pytest.approx(r, rel=1e-12) and got[1] == pytest.approx(j, rel=1e-12), (nnz, got, r, j)
    # an out-of-range index is flagged, as nomad_eval_rmse rejects it
    bad_row = tr[:100].clone()
    bad_row[5] = prob.m
    model.evaluate_noalloc(bad_row, tc[:100], tv[:100], out)
    torch.cuda.synchronize()
    assert out[2].item() == 1.0
    with pytest.raises(nm.NomadError):
        model.evaluate(bad_row, tc[:100], tv[:100])
    # no entries: RMSE is NaN, J is 0
    model.evaluate_noalloc(tr[:0], tc[:0], tv[:0], out)
    torch.cuda.synchronize()
    assert np.isnan(out[0].item()) and out[1].item() == 0.0 and out[2].item() == 0.0
    model.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    prob = synth.small_case(200, 100, 2_000, seed=62, k=8, test_frac=0.1)
    hp = prob.hp
    W0, H0 = synth.init_factors(prob.m, prob.n, hp["k"], 62)
    model = nm.Nomad(prob.m, prob.n, prob.row, prob.col, prob.val, W0, H0, k=hp["k"], lam=hp["lam"],
                     alpha=hp["alpha"], beta=hp["beta"], gamma=hp["gamma"], workers=4, seed=3)
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    lib = nm.load()
    # only the size is looked at: the arrays are never read
    rc = lib.nomad_eval_rmse_noalloc(model.ctx, 134_217_729, out.data_ptr(), out.data_ptr(), out.data_ptr(),
                                     out.data_ptr())
    assert rc == nm.NOMAD_EINVAL and b"exceeds" in lib.nomad_last_error(model.ctx)
    model.close()
