"""The device-side batched entry point (pwa_nll_batch_async): same kernels and
launch configuration as pwa_nll_batch, so the results must agree bit for bit;
it refuses to run before a synchronous call has prepared its workspace, and
replays of a captured graph must match fresh synchronous evaluations."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

PWA_E_STATE = 5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _real(Vs):
    v = np.empty((Vs.shape[0], 2 * Vs.shape[1]))
    v[:, 0::2], v[:, 1::2] = Vs.real, Vs.imag
    return v


@pytest.mark.parametrize("mode", ["stream", "gram"])
def test_batch_async_matches_sync(mode):
    import torch

    import paper_1108_5882_amd as pwa
    k, nv = 16, 40
    s = synth.make_sample(2, n_data=3001, n_mc=9007, k=k, seed=21)
    Vs = synth.eval_vectors(2, nv, k, seed=21)
    st = torch.cuda.Stream()
    with pwa.Context(0, "f32", stream=st) as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        c.set_mc_mode(mode, False)
        Vd = torch.from_numpy(_real(Vs)).cuda()
        out = torch.zeros(nv, 2 * k + 2, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        # matrix-core splits need the workspace of a synchronous call first
        for split in (2, 3):
            with pytest.raises(pwa.PwaError) as ei:
                c.nll_batch_async(Vd, out, split=split)
            assert ei.value.status == PWA_E_STATE
        for split in (0, 2, 3):
            nll, g = c.nll_batch(Vs, split=split)
            out.zero_()
            torch.cuda.synchronize()
            c.nll_batch_async(Vd, out, split=split)
            st.synchronize()
            o = out.cpu().numpy()
            _say(f"  {mode} split {split}: max |dnll| {np.max(np.abs(o[:, 0] - nll)):.1e}")
            assert np.array_equal(o[:, 0], nll), (mode, split)
            assert np.array_equal(o[:, 1:2 * k + 1], g), (mode, split)
            assert np.all(o[:, 2 * k + 1] == 0)
        # fewer vectors than prepared: still allowed, same results as a fresh sync call
        nll3, g3 = c.nll_batch(Vs[:7], split=3)
        out7 = torch.zeros(7, 2 * k + 2, dtype=torch.float64, device="cuda")
        c.nll_batch_async(Vd[:7].contiguous(), out7, split=3)
        st.synchronize()
        assert np.array_equal(out7.cpu().numpy()[:, 0], nll3)
        # a new sample invalidates the prepared inputs
        c.set_amplitudes("data", s.A_data[:2000])
        with pytest.raises(pwa.PwaError) as ei:
            c.nll_batch_async(Vd, out, split=2)
        assert ei.value.status == PWA_E_STATE


def test_batch_async_graph_replays():
    import torch

    import paper_1108_5882_amd as pwa
    k, nv = 32, 24
    s = synth.make_sample(2, n_data=4097, n_mc=8191, k=k, seed=22)
    Vs = synth.eval_vectors(2, 4 * nv, k, seed=22)
    st = torch.cuda.Stream()
    with pwa.Context(0, "f32", stream=st) as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        c.nll_batch(Vs[:nv], split=3)                 # prepares the workspace
        Vd = torch.from_numpy(_real(Vs[:nv])).cuda()
        out = torch.zeros(nv, 2 * k + 2, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            c.nll_batch_async(Vd, out, split=3)
        for r in range(4):
            batch = Vs[r * nv:(r + 1) * nv]
            with torch.cuda.stream(st):
                Vd.copy_(torch.from_numpy(_real(batch)))
                g.replay()
            st.synchronize()
            o = out.cpu().numpy()
            nll, gr = c.nll_batch(batch, split=3)      # eager work between replays
            _say(f"  replay {r}: max |dnll| {np.max(np.abs(o[:, 0] - nll)):.1e}")
            assert np.array_equal(o[:, 0], nll), r
            assert np.array_equal(o[:, 1:2 * k + 1], gr), r
