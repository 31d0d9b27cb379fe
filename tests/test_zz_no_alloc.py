"""The allocation-free entry point (ba_solve_noalloc) against ba_solve: same
batch, same configuration, two calls in a row on one GPU (the second smaller,
so the static workspace holds the first call's contents), each compared with
a handle's ba_solve to the FP64 / FP32 parity bar (bitwise here: the chunking
and the kernels are the same)."""
import numpy as np
import pytest
import torch

from paper_2208_04726_amd import native, synth
from paper_2208_04726_amd.solver import Solver, capacities_for, make_batch, solve_noalloc

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with_handle(wins, precision):
    b = make_batch(wins, precision)
    s = Solver(precision=precision, **capacities_for(wins))
    po, do = s.solve(b)
    torch.cuda.synchronize()
    st = s.status()
    s.close()
    return b, po.cpu().numpy(), do.cpu().numpy(), st


@pytest.mark.parametrize("precision,first,second", [
    ("fp32", [synth.method_scale_window(0), synth.method_scale_window(1), synth.serving_window(3)],
     [synth.serving_window(7)]),
    ("fp64", [synth.plain_fp64_window(i) for i in range(6)], [synth.plain_fp64_window(9)]),
])
def test_noalloc_matches_solve_twice(precision, first, second):
    _need_gpu()
    for wins in (first, second):
        print(f"{precision}: {len(wins)} windows, {sum(w.kk.shape[0] for w in wins)} edges", flush=True)
        b, po_ref, do_ref, st_ref = _with_handle(wins, precision)
        po, do, st = solve_noalloc(b, precision)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == st_ref).all() and (st_ref == 0).all()
        po, do = po.cpu().numpy(), do.cpu().numpy()
        print(f"  max |pose diff| {np.abs(po - po_ref).max():.2e}, max |depth diff| {np.abs(do - do_ref).max():.2e}")
        assert np.array_equal(po, po_ref) and np.array_equal(do, do_ref)


def test_noalloc_rejects_oversize_batch_before_enqueueing():
    """64 windows of 22 x 96 need more than the 64 MiB static workspace:
    BA_E_CAPACITY, and the outputs keep their sentinel."""
    _need_gpu()
    w = synth.method_scale_window(0)
    b = make_batch([w] * 64, "fp32")
    F, P, _ = b.totals
    po = torch.full((F, 7), -7.0, dtype=torch.float64, device="cuda")
    do = torch.full((P,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(native.BAError) as e:
        solve_noalloc(b, "fp32", poses_out=po, depth_out=do)
    assert e.value.code == native.BA_E_CAPACITY
    torch.cuda.synchronize()
    assert (po == -7.0).all() and (do == -7.0).all()
