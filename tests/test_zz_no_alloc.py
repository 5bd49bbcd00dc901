"""The entry point that allocates nothing (cg_process_batch_static) against
cg_process_batch_ex on the same frames: its workspace is the library's fixed
scratch array instead of the plan's, the kernels are the same, so every
output is bit-identical.  Two calls in a row, the second with a smaller
batch (the array keeps the first call's contents), for the cold start and
the learned warm start; a batch beyond the array and a matrix-core form are
refused before any work is enqueued."""

import os
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12988_amd as cg  # noqa: E402

DEV = torch.device("cuda:0")
WEIGHTS = os.path.join(os.path.dirname(cg.__file__), "data", "warmstart_learned.npz")
SCRATCH = 64 << 20


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _outs(nf):
    return (torch.empty((nf, 4), dtype=torch.float32, device=DEV),
            torch.empty((nf,), dtype=torch.int32, device=DEV),
            torch.empty((nf,), dtype=torch.int32, device=DEV),
            torch.empty((nf,), dtype=torch.float32, device=DEV))


@pytest.mark.parametrize("form", ["cold", "warm"])
def test_static_matches_process_batch_ex_twice(form):
    spec = synth.spec_paper_rate() if form == "cold" else synth.spec_learned()
    bt = synth.make_batch(spec, 40000, seed=21)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins).astype(np.float32)
    plan = cg.Plan(spec.n, spec.fs, spec.bins, ref)
    flags = cg.FIT_COLD
    if form == "warm":
        if not os.path.exists(WEIGHTS):
            pytest.skip("trained weights not built")
        d = np.load(WEIGHTS)
        plan.set_mlp(d["params"], d["out_mean"], d["out_std"], float(d["noise_floor"]))
        flags = cg.FIT_WARM_MLP
    assert plan.workspace_bytes(40000) <= SCRATCH
    fr_all = torch.from_numpy(bt.frames).to(DEV)
    for nf in (40000, 2999):
        _say(f"static entry point, {form}, {nf} frames")
        fr = fr_all[:nf]
        a = _outs(nf)
        plan.process_static(fr, *a, flags=flags)
        b = plan.process(fr, params=torch.empty((nf, 4), dtype=torch.float32, device=DEV),
                         iters=torch.empty((nf,), dtype=torch.int32, device=DEV),
                         status=torch.empty((nf,), dtype=torch.int32, device=DEV),
                         chi2=torch.empty((nf,), dtype=torch.float32, device=DEV),
                         flags=flags, want=())
        torch.cuda.synchronize()
        for x, name in zip(a, ("params", "iters", "status", "chi2")):
            assert torch.equal(x, b[name]), (form, nf, name)
        st = a[2].cpu().numpy()
        _say(f"  identical; statuses {np.bincount(st, minlength=4).tolist()}")
    plan.close()


def test_static_refuses_what_it_cannot_do_without_allocating():
    spec = synth.spec_paper_rate()
    plan = cg.Plan(spec.n, spec.fs, spec.bins, np.ones(spec.k, dtype=np.float32))
    big = 1
    while plan.workspace_bytes(big) <= SCRATCH:
        big *= 2
    assert big > 65536                     # a whole paper-rate batch fits
    fr = torch.zeros((big, spec.n), dtype=torch.int16, device=DEV)
    params = torch.full((big, 4), -7.0, dtype=torch.float32, device=DEV)
    with pytest.raises(cg.CombGpuError) as ex:
        plan.process_static(fr, params)
    assert ex.value.status == -7           # CG_ERR_WORKSPACE
    small = fr[:64]
    with pytest.raises(cg.CombGpuError):
        plan.process_static(small, params[:64], flags=cg.DFT_MFMA_BF16X3)
    with pytest.raises(cg.CombGpuError):
        plan.process_static(small, params[:64], flags=cg.FIT_WARM_MLP)   # no network set
    torch.cuda.synchronize()
    assert torch.all(params == -7.0)      # nothing was enqueued
    plan.close()
