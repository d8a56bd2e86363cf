"""Scratch memory through the caller's allocator (cg_allocator): the Python binding
passes one backed by PyTorch's caching allocator, and a failing allocation anywhere in
a forward or backward call returns CG_ERR_OUT_OF_MEMORY, frees what the call held and
leaves the library ready for the next call."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_13397_amd import synth
from parity import compare_image

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _counting_allocator(fail_at=None):
    """A torch-backed allocator that records its live blocks and fails its fail_at-th
    allocation (1-based; None: never)."""
    from paper_2609_13397_amd import render as R

    class Counting(R.TorchAllocator):
        def __init__(self):
            super().__init__()
            self.calls = 0
            self.live = set()

        def allocate(self, nbytes, stream):
            self.calls += 1
            if self.calls == fail_at:
                raise MemoryError("planted failure")
            p = super().allocate(nbytes, stream)
            self.live.add(p)
            return p

        def release(self, ptr):
            self.live.discard(ptr)
            super().release(ptr)

    return Counting()


def test_scratch_comes_from_torch_and_is_returned():
    import torch
    from paper_2609_13397_amd import render as R
    scene, cam = synth.tiny_config()
    sc = R.Scene.from_numpy(scene)
    _say("torch-owned scratch")
    a = _counting_allocator()
    rgba, info, _ = R.render_forward(sc, [cam], R.RenderOpts(), allocator=a)
    torch.cuda.synchronize()
    assert a.calls >= 2 and not a.live  # every block of an inference call is freed by its end
    img = rgba.view(cam["crop"][3], cam["crop"][2], 4).cpu().numpy().astype(np.float64)
    nfail, worst, det = compare_image(img, O.render(scene, cam, O.Opts(), with_alt=True))
    assert nfail == 0, det
    _, _, st = R.render_forward(sc, [cam], R.RenderOpts(), need_state=True, allocator=a)
    held = len(a.live)
    assert held >= 2  # the training state keeps its scratch
    R.render_backward(st, torch.ones_like(rgba), sc)
    torch.cuda.synchronize()
    assert len(a.live) == held  # the backward's own scratch is returned
    st.release()
    assert not a.live


@pytest.mark.parametrize("fail_at", [1, 2])
def test_forward_allocation_failure_is_out_of_memory(fail_at):
    import torch
    from paper_2609_13397_amd import _lib
    from paper_2609_13397_amd import render as R
    scene, cam = synth.tiny_config()
    sc = R.Scene.from_numpy(scene)
    _say(f"forward allocation failure at call {fail_at}")
    ok, _, _ = R.render_forward(sc, [cam], R.RenderOpts())
    ok = ok.clone()
    for need_state in (False, True):
        a = _counting_allocator(fail_at)
        with pytest.raises(_lib.CgError) as ei:
            R.render_forward(sc, [cam], R.RenderOpts(), need_state=need_state, allocator=a)
        torch.cuda.synchronize()
        assert ei.value.status == -3, ei.value  # CG_ERR_OUT_OF_MEMORY
        assert a.calls == fail_at and not a.live
        # the next call on the same allocator (no more failures) renders the same image
        again, _, st = R.render_forward(sc, [cam], R.RenderOpts(), need_state=need_state, allocator=a)
        torch.cuda.synchronize()
        assert torch.equal(again, ok)
        if st is not None:
            st.release()
        assert not a.live


def test_backward_allocation_failure_is_out_of_memory():
    import torch
    from paper_2609_13397_amd import _lib
    from paper_2609_13397_amd import render as R
    scene, cam = synth.tiny_config()
    sc = R.Scene.from_numpy(scene)
    _say("backward allocation failure")
    probe = _counting_allocator()
    _, _, st = R.render_forward(sc, [cam], R.RenderOpts(), need_state=True, allocator=probe)
    n_fwd = probe.calls
    G = torch.from_numpy(synth.seeded_image((cam["crop"][3] * cam["crop"][2], 4), seed=3)).cuda()
    ref = R.render_backward(st, G, sc)
    torch.cuda.synchronize()
    st.release()
    a = _counting_allocator(n_fwd + 1)
    _, _, st = R.render_forward(sc, [cam], R.RenderOpts(), need_state=True, allocator=a)
    held = set(a.live)
    with pytest.raises(_lib.CgError) as ei:
        R.render_backward(st, G, sc)
    torch.cuda.synchronize()
    assert ei.value.status == -3 and a.live == held
    g = R.render_backward(st, G, sc)  # the state is intact: the retry succeeds
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(g[k], ref[k]), k
    st.release()
    assert not a.live
