"""Pins of the oracle's chunked (multi-threaded) form against the plain oracle.

The chunked form sums fixed chunks of events in event order and adds the chunk
sums in chunk order (the precision remark of Section 2: double-precision tree
sums), so
  * its result is bitwise the same for every thread count;
  * a sample within one chunk gives bitwise the plain oracle's result (one
    chunk is the plain sum, and adding it to zero is exact);
  * across chunks it agrees with the plain oracle to rounding (1e-14 of the
    term scale), in both likelihood forms, with weights and N_gen.
"""
import numpy as np
import pytest

import oracle
import synth


def _case(seed, nd, nm, k, weighted=True):
    g = np.random.default_rng(seed)
    Ad = synth.random_amplitudes(g, nd, k, np.complex128)
    Am = synth.random_amplitudes(g, nm, k, np.complex128)
    w = g.uniform(0.2, 3.0, nm) if weighted else None
    return Ad, Am, synth.draw_v(g, 1, k)[0], w


@pytest.mark.parametrize("extended", [False, True])
def test_thread_count_independent(extended):
    Ad, Am, V, w = _case(1, 140_001, 200_003, 7)
    ref = oracle.nll_grad_chunked(Ad, Am, V, w=w, n_gen=250_000, extended=extended, threads=1)
    for t in (2, 3, 8):
        r = oracle.nll_grad_chunked(Ad, Am, V, w=w, n_gen=250_000, extended=extended, threads=t)
        assert r[0] == ref[0] and np.array_equal(r[1], ref[1]), t


def test_one_chunk_equals_plain_oracle():
    Ad, Am, V, w = _case(2, 5_001, 60_000, 12)
    a = oracle.nll_grad(Ad, Am, V, w=w, n_gen=70_000)
    b = oracle.nll_grad_chunked(Ad, Am, V, w=w, n_gen=70_000, threads=4)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("extended", [False, True])
def test_many_chunks_agree_with_plain_oracle(extended):
    Ad, Am, V, w = _case(3, 200_017, 330_001, 16)
    nll, grad, p = oracle.nll_grad(Ad, Am, V, w=w, extended=extended, parts=True)
    nll_c, grad_c, pc = oracle.nll_grad_chunked(Ad, Am, V, w=w, extended=extended, threads=4, parts=True)
    I = oracle.intensity(Ad, V)
    scale = float(np.sum(np.abs(np.log(I)))) + Ad.shape[0] * abs(np.log(p["s_raw"] / Am.shape[0])) + p["s_raw"]
    assert abs(nll - nll_c) / scale < 1e-14
    assert np.max(np.abs(grad - grad_c)) / np.max(np.abs(grad)) < 1e-12
    for key in ("GD", "HM"):
        assert np.max(np.abs(p[key] - pc[key])) / np.max(np.abs(p[key])) < 1e-13
