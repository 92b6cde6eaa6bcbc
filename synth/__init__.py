"""Seeded synthetic inputs for the partial-wave likelihood.

This module builds the inputs that both the FP64 oracle and the GPU library
consume: per-event complex decay amplitudes A_alpha(Omega) for data and Monte
Carlo (MC) samples, optional MC weights, and production-amplitude vectors V.
It computes no part of the likelihood, its gradient or its normalisation.

Physics stand-in (the paper's worked channel is J/psi -> gamma X, X -> K+K-,
Section 2; its data and resonance parametrisation are not public here):

* kinematics Omega = (m, cos theta) with m the K+K- mass in [0.99, 3.0] GeV and
  cos theta in [-1, 1];
* each wave alpha is a fixed-width relativistic Breit-Wigner in m times a
  spherical harmonic Y_J^0(cos theta):
      A_alpha = 1 / (m_alpha^2 - m^2 - i m_alpha Gamma_alpha) * Y_{J_alpha}^0(cos theta)
* MC events are generated flat in (m, cos theta); the optional weighted variant
  draws m from a resonance-peaked density and weights events back to a flat
  distribution (the footnote on MC generation in Section 2);
* data events are drawn by accept-reject from the model density at a fixed
  "true" production vector.  The acceptance density is the physical event
  density of the model; it is used for nothing but drawing this sample.

Every array is a deterministic function of (config, scale, seed).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_ROOT = 11085882
M_LO, M_HI = 0.99, 3.0          # K+K- mass range in GeV
X_LO, X_HI = -1.0, 1.0          # cos(theta) range

# Random streams, one per independent draw, so that changing one size never
# shifts another draw.
_S_WAVES, _S_VTRUE, _S_MC, _S_DATA, _S_VEVAL, _S_PILOT, _S_NET = range(7)

CHUNK = 1 << 18


def rng_for(cfg: int, seed: int, stream: int) -> np.random.Generator:
    """PCG64 generator keyed by (root, config, seed, stream)."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([SEED_ROOT, int(cfg), int(seed), int(stream)])))


@dataclasses.dataclass
class Waves:
    mass: np.ndarray    # GeV, [K]
    width: np.ndarray   # GeV, [K]
    J: np.ndarray       # spin, [K]

    @property
    def k(self) -> int:
        return int(self.mass.shape[0])


# ---------------------------------------------------------------- amplitudes
def _legendre(J: int, x: np.ndarray) -> np.ndarray:
    """Legendre polynomial P_J by Bonnet's recurrence."""
    p0 = np.ones_like(x)
    if J == 0:
        return p0
    p1 = x.copy()
    for n in range(1, J):
        p0, p1 = p1, ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
    return p1


def y_j0(J: int, x: np.ndarray) -> np.ndarray:
    """Spherical harmonic Y_J^0(cos theta) = sqrt((2J+1)/(4 pi)) P_J(cos theta)."""
    return math.sqrt((2 * J + 1) / (4.0 * math.pi)) * _legendre(J, x)


def breit_wigner(m: np.ndarray, mass: float, width: float) -> np.ndarray:
    """Fixed-width relativistic Breit-Wigner 1/(M^2 - m^2 - i M Gamma)."""
    return 1.0 / ((mass * mass - m * m) - 1j * (mass * width))


def amplitudes(m: np.ndarray, x: np.ndarray, waves: Waves,
               out_dtype=np.complex128) -> np.ndarray:
    """A[n, K] with A[i, alpha] = BW_alpha(m_i) * Y_{J_alpha}^0(x_i)."""
    n, k = m.shape[0], waves.k
    ys = {int(J): y_j0(int(J), x) for J in np.unique(waves.J)}
    m2 = m * m
    # build wave-major (contiguous per wave), transpose once at the end
    re = np.empty((k, n))
    im = np.empty((k, n))
    for a in range(k):
        M, G = float(waves.mass[a]), float(waves.width[a])
        d = M * M - m2                       # BW = (d + i M G) / (d^2 + (M G)^2)
        inv = 1.0 / (d * d + (M * G) ** 2)
        y = ys[int(waves.J[a])]
        re[a] = d * inv * y
        im[a] = (M * G) * inv * y
    out = np.empty((n, k), dtype=out_dtype)
    out.real = re.T
    out.imag = im.T
    return out


# -------------------------------------------------------------- wave tables
def waves_for(cfg: int, k: Optional[int] = None, seed: int = 0, fit: int = 0) -> Waves:
    """Resonance table of a configuration.

    cfg 0: the K=4 table (1.5, 0.05, J=0), (1.7, 0.10, 2), (2.0, 0.15, 0),
    (2.3, 0.20, 2).  Otherwise masses U[1.2, 2.8] GeV, widths U[0.03, 0.3] GeV,
    J cycling through (0, 2, 4).
    """
    if cfg == 0:
        return Waves(np.array([1.5, 1.7, 2.0, 2.3]), np.array([0.05, 0.10, 0.15, 0.20]),
                     np.array([0, 2, 0, 2]))
    if k is None:
        k = {1: 16, 2: 32, 4: 16}[cfg]
    g = rng_for(cfg, seed, _S_WAVES * 1000 + fit)
    mass = g.uniform(1.2, 2.8, k)
    width = g.uniform(0.03, 0.3, k)
    J = np.array([(0, 2, 4)[a % 3] for a in range(k)])
    return Waves(mass, width, J)


# --------------------------------------------------------------- V vectors
def draw_v(g: np.random.Generator, nv: int, k: int) -> np.ndarray:
    """Production vectors: |V| log-uniform in [0.1, 10], phase uniform in [0, 2 pi)."""
    mag = 10.0 ** g.uniform(-1.0, 1.0, (nv, k))
    ph = g.uniform(0.0, 2.0 * math.pi, (nv, k))
    return mag * np.exp(1j * ph)


def v_true(cfg: int, k: int, seed: int = 0, fit: int = 0) -> np.ndarray:
    """The production vector the data sample is drawn at, with V_0 real and positive."""
    v = draw_v(rng_for(cfg, seed, _S_VTRUE * 1000 + fit), 1, k)[0]
    return v * np.exp(-1j * np.angle(v[0]))


def eval_vectors(cfg: int, nv: int, k: int, seed: int = 0, stream: int = 0) -> np.ndarray:
    """nv evaluation vectors drawn from the V law (independent of the data)."""
    return draw_v(rng_for(cfg, seed, _S_VEVAL * 1000 + stream), nv, k)


# -------------------------------------------------------------- kinematics
def _peaked_m(g: np.random.Generator, n: int, waves: Waves):
    """m from q(m) = 1/2 flat + 1/2 equal mixture of Cauchy peaks truncated to the range.

    Returns (m, q(m)); a flat-sample weight is then (1/(M_HI-M_LO)) / q(m).
    """
    span = M_HI - M_LO
    k = waves.k
    flat = g.random(n) < 0.5
    comp = g.integers(0, k, n)
    u = g.random(n)
    mu = waves.mass[comp]
    gam = 0.5 * waves.width[comp]
    lo = np.arctan((M_LO - mu) / gam)
    hi = np.arctan((M_HI - mu) / gam)
    m_peak = mu + gam * np.tan(lo + u * (hi - lo))
    m = np.where(flat, M_LO + span * u, m_peak)
    # mixture density; a Cauchy peak truncated to [lo, hi] has density
    # g / ((m - mu)^2 + g^2) / (atan((hi - mu)/g) - atan((lo - mu)/g))
    dens = np.zeros(n)
    for a in range(k):
        ga = 0.5 * waves.width[a]
        za = (np.arctan((M_HI - waves.mass[a]) / ga) - np.arctan((M_LO - waves.mass[a]) / ga))
        dens += ga / ((m - waves.mass[a]) ** 2 + ga * ga) / za
    q = 0.5 / span + 0.5 * dens / k
    return m, q


def mc_kinematics(g: np.random.Generator, n: int, waves: Waves, weighted: bool):
    x = g.uniform(X_LO, X_HI, n)
    if not weighted:
        return g.uniform(M_LO, M_HI, n), x, None
    m, q = _peaked_m(g, n, waves)
    w = (1.0 / (M_HI - M_LO)) / q
    return m, x, w


def _event_density(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Physical event density of the model at production vector v (used only to
    accept or reject candidate data events)."""
    s = A @ v
    return s.real * s.real + s.imag * s.imag


def _proposal_table(g: np.random.Generator, waves: Waves, v: np.ndarray, nbins: int = 512,
                    per_bin: int = 128):
    """Piecewise-constant envelope h(m) over mass bins, from a pilot scan.

    h_b = 2 x the largest model density seen in bins b-1..b+1, floored at
    1e-3 of the maximum so every bin stays reachable.
    """
    edges = np.linspace(M_LO, M_HI, nbins + 1)
    width = edges[1] - edges[0]
    b = np.repeat(np.arange(nbins), per_bin)
    m = edges[b] + width * g.random(b.shape[0])
    x = g.uniform(X_LO, X_HI, b.shape[0])
    f = _event_density(amplitudes(m, x, waves), v).reshape(nbins, per_bin).max(axis=1)
    h = np.maximum(np.maximum(f, np.roll(f, 1)), np.roll(f, -1))
    h[0] = max(f[0], f[1])
    h[-1] = max(f[-1], f[-2])
    h = 2.0 * np.maximum(h, 1e-3 * h.max())
    return edges, h


def data_kinematics(g_pilot: np.random.Generator, g: np.random.Generator, n: int,
                    waves: Waves, v: np.ndarray):
    """Accept-reject draw of n events with density proportional to the model at v.

    Candidates: a mass bin chosen with probability proportional to the envelope
    h_b, m uniform in the bin, cos theta uniform.  A candidate with model
    density f is kept with probability f / h_b.  If any candidate has f > h_b
    the envelope doubles and the draw restarts from the same generator state,
    so the result stays deterministic and follows the model density wherever
    the envelope bounds it.
    """
    if n == 0:
        return np.empty(0), np.empty(0)
    edges, h = _proposal_table(g_pilot, waves, v)
    width = edges[1] - edges[0]
    state = g.bit_generator.state
    while True:
        g.bit_generator.state = state
        cdf = np.cumsum(h) / h.sum()
        ms, xs, got, ok = [], [], 0, True
        while got < n:
            b = np.minimum(np.searchsorted(cdf, g.random(CHUNK), side="right"), h.shape[0] - 1)
            m = edges[b] + width * g.random(CHUNK)
            x = g.uniform(X_LO, X_HI, CHUNK)
            f = _event_density(amplitudes(m, x, waves), v)
            env = h[b]
            if np.any(f > env):
                ok = False
                break
            keep = g.random(CHUNK) * env < f
            ms.append(m[keep])
            xs.append(x[keep])
            got += int(keep.sum())
        if ok:
            return np.concatenate(ms)[:n], np.concatenate(xs)[:n]
        h = 2.0 * h


# ---------------------------------------------------------------- samples
@dataclasses.dataclass
class Sample:
    waves: Waves
    A_data: np.ndarray            # [N_D, K] complex64 (FP32 configs) or complex128
    A_mc: np.ndarray              # [N_MC, K]
    w_mc: Optional[np.ndarray]    # [N_MC] float, or None for unit weights
    n_gen: float                  # MC normalisation count (>= N_MC)
    V_true: np.ndarray            # [K] complex128, the vector the data were drawn at

    @property
    def k(self) -> int:
        return self.waves.k


# Sizes of the five workloads: (N_data, N_MC, K, precision).
CONFIGS = {
    0: dict(n_data=10_000, n_mc=100_000, k=4, dtype=np.complex128),
    1: dict(n_data=1_000_000, n_mc=5_000_000, k=16, dtype=np.complex64),
    2: dict(n_data=2_000_000, n_mc=10_000_000, k=32, dtype=np.complex64),
    4: dict(n_data=1_000_000, n_mc=5_000_000, k=16, dtype=np.complex64),
}


def _amps_chunked(m, x, waves, dtype):
    out = np.empty((m.shape[0], waves.k), dtype=dtype)
    for s in range(0, m.shape[0], CHUNK):
        out[s:s + CHUNK] = amplitudes(m[s:s + CHUNK], x[s:s + CHUNK], waves, np.complex128)
    return out


def make_sample(cfg: int, scale: float = 1.0, seed: int = 0, weighted: bool = False,
                n_data: Optional[int] = None, n_mc: Optional[int] = None,
                k: Optional[int] = None, dtype=None, fit: int = 0,
                accept_fraction: float = 1.0) -> Sample:
    """Build the data and MC amplitude arrays of a workload.

    cfg selects the wave table and V law (0..4 as in ``CONFIGS``; cfg 3 is the
    uneven multi-fit family and needs explicit n_data, n_mc, k and ``fit``).
    ``scale`` shrinks both sample sizes.  ``accept_fraction`` < 1 keeps only
    that fraction of generated MC rows (detector acceptance) while n_gen stays
    the generated count.
    """
    base = CONFIGS.get(cfg, {})
    nd = int(round((n_data if n_data is not None else base["n_data"]) * (scale if n_data is None else 1)))
    nm = int(round((n_mc if n_mc is not None else base["n_mc"]) * (scale if n_mc is None else 1)))
    k = k if k is not None else base["k"]
    dtype = dtype if dtype is not None else base.get("dtype", np.complex64)
    waves = waves_for(cfg, k=k, seed=seed, fit=fit)
    vt = v_true(cfg, waves.k, seed=seed, fit=fit)
    g_mc = rng_for(cfg, seed, _S_MC * 1000 + fit)
    m, x, w = mc_kinematics(g_mc, nm, waves, weighted)
    n_gen = float(nm)
    if accept_fraction < 1.0:
        keep = g_mc.random(nm) < accept_fraction
        m, x = m[keep], x[keep]
        w = None if w is None else w[keep]
    A_mc = _amps_chunked(m, x, waves, dtype)
    md, xd = data_kinematics(rng_for(cfg, seed, _S_PILOT * 1000 + fit),
                             rng_for(cfg, seed, _S_DATA * 1000 + fit), nd, waves, vt)
    A_data = _amps_chunked(md, xd, waves, dtype)
    if w is not None:
        w = w.astype(np.float32 if dtype == np.complex64 else np.float64)
    return Sample(waves, A_data, A_mc, w, n_gen, vt)


@dataclasses.dataclass
class KinSample:
    """Per-event kinematics of a workload: (m_KK, cos theta) as FP32 pairs."""
    waves: Waves
    mx_data: np.ndarray        # [N_data, 2] float32
    mx_mc: np.ndarray          # [N_MC, 2] float32
    w_mc: Optional[np.ndarray]
    n_gen: float
    V_true: np.ndarray

    @property
    def k(self) -> int:
        return self.waves.k

    @property
    def res(self) -> np.ndarray:
        """(m_a, Gamma_a) interleaved, FP64."""
        r = np.empty(2 * self.k)
        r[0::2], r[1::2] = self.waves.mass, self.waves.width
        return r


def make_kin_sample(cfg: int, scale: float = 1.0, seed: int = 0, weighted: bool = False,
                    n_data: Optional[int] = None, n_mc: Optional[int] = None, k: Optional[int] = None,
                    fit: int = 0) -> KinSample:
    """The kinematics make_sample draws (same seeds, same accept-reject of the data
    at V_true), kept as FP32 (m, cos theta) pairs instead of amplitude rows."""
    base = CONFIGS.get(cfg, {})
    nd = int(round((n_data if n_data is not None else base["n_data"]) * (scale if n_data is None else 1)))
    nm = int(round((n_mc if n_mc is not None else base["n_mc"]) * (scale if n_mc is None else 1)))
    k = k if k is not None else base["k"]
    waves = waves_for(cfg, k=k, seed=seed, fit=fit)
    vt = v_true(cfg, waves.k, seed=seed, fit=fit)
    m, x, w = mc_kinematics(rng_for(cfg, seed, _S_MC * 1000 + fit), nm, waves, weighted)
    md, xd = data_kinematics(rng_for(cfg, seed, _S_PILOT * 1000 + fit),
                             rng_for(cfg, seed, _S_DATA * 1000 + fit), nd, waves, vt)
    mx_mc = np.stack([m, x], axis=1).astype(np.float32)
    mx_data = np.stack([md, xd], axis=1).astype(np.float32)
    return KinSample(waves, mx_data, mx_mc, None if w is None else w.astype(np.float32), float(nm), vt)


def multifit_table(nfits: int = 64, seed: int = 0):
    """The uneven multi-fit family: per fit (N_data, K, N_MC = 5 N_data).

    N_data log-uniform in [1e4, 1e6], K uniform in {4..48}.
    """
    g = rng_for(3, seed, 99)
    nd = np.round(10.0 ** g.uniform(4.0, 6.0, nfits)).astype(np.int64)
    ks = g.integers(4, 49, nfits)
    return [(int(a), int(b), int(5 * a)) for a, b in zip(nd, ks)]


def gaussian_integer_amplitudes(g: np.random.Generator, n: int, k: int, bound: int = 4,
                                dtype=np.complex64) -> np.ndarray:
    """Amplitudes with integer real and imaginary parts in [-bound, bound]."""
    re = g.integers(-bound, bound + 1, (n, k))
    im = g.integers(-bound, bound + 1, (n, k))
    return (re + 1j * im).astype(dtype)


def random_amplitudes(g: np.random.Generator, n: int, k: int, dtype=np.complex64) -> np.ndarray:
    """Unstructured complex normal amplitudes (for shape and edge-case tests)."""
    return (g.standard_normal((n, k)) + 1j * g.standard_normal((n, k))).astype(dtype)


# --------------------------------------------------------- surrogate inputs
def mlp_init(n_in: int, hidden: int, seed: int = 0) -> np.ndarray:
    """Initial parameters of an n_in -> hidden -> hidden -> 1 network, FP32, in the
    layout [W1 (hidden x n_in) | b1 | W2 (hidden x hidden) | b2 | w3 | b3].

    Every weight and bias of a layer with fan-in f is uniform in [-1/sqrt(f),
    1/sqrt(f)] (the default initialisation of a PyTorch linear layer).
    """
    g = rng_for(4, seed, _S_NET)
    parts = []
    for fan_in, shape in ((n_in, (hidden, n_in)), (n_in, (hidden,)), (hidden, (hidden, hidden)),
                          (hidden, (hidden,)), (hidden, (hidden,)), (hidden, (1,))):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(g.uniform(-b, b, shape).ravel())
    return np.concatenate(parts).astype(np.float32)


def permutations(n: int, epochs: int, batch: int, seed: int = 0) -> np.ndarray:
    """Mini-batch order for `epochs` passes over n rows: each epoch a fresh
    random permutation cut into floor(n / batch) batches (the remainder is
    left out of that epoch).  int32, epochs * floor(n / batch) * batch entries."""
    g = rng_for(4, seed, _S_NET * 1000 + 1)
    per = (n // batch) * batch
    return np.concatenate([g.permutation(n)[:per] for _ in range(epochs)]).astype(np.int32)
