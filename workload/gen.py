"""Seeded input generators (numpy PCG64), all produced in fp64.

Matrices
--------
sym_gaussian(n, seed)        A = (G + G^T)/2, G_ij ~ N(0, 1)
herm_gaussian(n, seed)       A = (G + G^H)/2, Re G_ij, Im G_ij ~ N(0, 1/2)
haar_spectrum(n, sq, sl)     A = Q diag(lambda) Q^T, Q Haar orthogonal (QR of a
                             Gaussian with diag(R) > 0), lambda ~ U[-1, 1]

Back-transformation inputs (boundary layout of the reflectors)
--------------------------------------------------------------
reflector_layout(n, b)       sweep, chase step, row start and length per slot
synthetic_reflectors(...)    random unit-norm-preserving Householder reflectors
                             laid out as the band->tridiagonal chase emits them
gaussian_block(n, nev, ...)  a dense n x nev block standing in for eigenvectors
device_reflectors, device_block   the same drawn on the GPU with torch (served
                             stream throughput runs)
synthetic_stage1(n, b, ...)  first-stage (full -> band) reflectors in the layout
                             of the band -> full back-transformation

Workload sizes and traces
-------------------------
batched_sizes, scf_sequence_sizes, scf_trace (Poisson arrivals, fp32 share or a
switch from fp32 to fp64 at a given SCF step)

The synthetic reflectors have the structure of the real ones: v[0] = 1, the
other L-1 entries of size about 1/sqrt(b), zero padding past L, and a tau that
makes H = I - tau v v^H exactly orthogonal / unitary up to the rounding of tau
(real: tau = 2/||v||^2, tau = 0 for L = 1 like LAPACK; complex:
tau = (1 - e^{i theta})/||v||^2).  The values a real bulge chase would produce
differ, the shapes, sizes, slot structure and magnitudes do not.
"""
import numpy as np

__all__ = [
    "synthetic_stage1",
    "sym_gaussian", "herm_gaussian", "haar_spectrum", "reflector_layout",
    "synthetic_reflectors", "gaussian_block", "to_dtype",
    "batched_sizes", "scf_sequence_sizes", "scf_trace",
    "device_reflectors", "device_block",
]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def sym_gaussian(n, seed):
    G = _rng(seed).standard_normal((n, n))
    return (G + G.T) / 2.0


def herm_gaussian(n, seed):
    g = _rng(seed)
    s = np.sqrt(0.5)
    G = g.standard_normal((n, n)) * s + 1j * (g.standard_normal((n, n)) * s)
    return (G + G.conj().T) / 2.0


def haar_spectrum(n, seed_q, seed_l):
    X = _rng(seed_q).standard_normal((n, n))
    Qh, R = np.linalg.qr(X)
    Qh = Qh * np.sign(np.diag(R))[None, :]
    lam = _rng(seed_l).uniform(-1.0, 1.0, n)
    A = (Qh * lam[None, :]) @ Qh.T
    return (A + A.T) / 2.0


def reflector_layout(n, b):
    """Per-slot (s, j, r, L) arrays in generation order (s, then j)."""
    if n < 2:
        z = np.zeros(0, dtype=np.int64)
        return z, z, z, z
    s = np.arange(n - 1, dtype=np.int64)
    J = (n - 1 - s + b - 1) // b
    off = np.concatenate([[0], np.cumsum(J)[:-1]])
    ss = np.repeat(s, J)
    jj = np.arange(int(J.sum()), dtype=np.int64) - np.repeat(off, J)
    rr = ss + 1 + jj * b
    LL = np.minimum(b, n - rr)
    return ss, jj, rr, LL


def synthetic_reflectors(n, b, complex_=False, seed=0, chunk=1 << 18):
    """Random Householder reflectors in the boundary layout.

    Returns (hh, tau): hh has shape (nrefl*b,), tau (nrefl,), fp64 or complex128.
    """
    _, _, _, LL = reflector_layout(n, b)
    N = LL.size
    g = _rng(seed)
    dt = np.complex128 if complex_ else np.float64
    hh = np.zeros((N, b), dtype=dt)
    tau = np.zeros(N, dtype=dt)
    col = np.arange(b)[None, :]
    sc = 1.0 / np.sqrt(b)
    for a in range(0, N, chunk):
        e = min(N, a + chunk)
        m = e - a
        if complex_:
            h = np.sqrt(0.5) * sc
            v = g.standard_normal((m, b)) * h + 1j * (g.standard_normal((m, b)) * h)
        else:
            v = g.standard_normal((m, b)) * sc
        v[:, 0] = 1.0
        v[col >= LL[a:e, None]] = 0.0
        nrm2 = np.sum(np.abs(v) ** 2, axis=1)
        if complex_:
            th = g.uniform(0.0, 2.0 * np.pi, m)
            t = (1.0 - np.exp(1j * th)) / nrm2
        else:
            t = 2.0 / nrm2
            t[LL[a:e] == 1] = 0.0
        hh[a:e] = v
        tau[a:e] = t
    return hh.reshape(-1), tau


def gaussian_block(n, nev, complex_=False, seed=0):
    """Dense n x nev column-major block, entries N(0, 1/n) (complex: each part
    N(0, 1/(2n))), the size of unit eigenvector entries."""
    g = _rng(seed)
    s = 1.0 / np.sqrt(n)
    if complex_:
        h = s * np.sqrt(0.5)
        Z = g.standard_normal((nev, n)) * h + 1j * (g.standard_normal((nev, n)) * h)
    else:
        Z = g.standard_normal((nev, n)) * s
    return Z.T  # F-ordered view: column c is contiguous


def to_dtype(x, name):
    """Round fp64 / complex128 inputs to the request precision."""
    return {"r64": np.float64, "r32": np.float32, "c64": np.complex128}[name](x) \
        if np.isscalar(x) else x.astype(
            {"r64": np.float64, "r32": np.float32, "c64": np.complex128}[name])


def batched_sizes(count=256, lo=200, hi=2000, seed=401):
    """Problem sizes of the batched workload: n_i ~ U{lo..hi}."""
    return _rng(seed).integers(lo, hi + 1, size=count)


def scf_sequence_sizes(count=64, lo=1000, hi=6000, seed=501):
    """Per-sequence sizes of the served SCF stream: n_q ~ U{lo..hi}."""
    return _rng(seed).integers(lo, hi + 1, size=count)


def scf_trace(nseq=64, steps=20, rate=200.0, p32=0.25, seed_arrivals=502, seed_dtypes=503,
              switch_step=None):
    """Arrival trace of the served SCF stream: nseq sequences of `steps` solves.

    A Poisson process of the given rate (requests per second) gives
    nseq*steps arrival times; request i belongs to sequence i % nseq as its
    step i // nseq (each sequence's solves arrive in order, and a solve is
    also held back until the sequence's previous solve has completed).  Each
    request is fp32 with probability p32, else fp64; with switch_step given
    instead, a sequence's steps before switch_step are fp32 and the rest fp64
    (single precision while the SCF cycle is far from convergence, double for
    the final steps, the switching of Kus et al., Sec. 5.2).  Returns
    (arrival seconds, sequence, step, is_fp32) arrays.
    """
    total = nseq * steps
    t = np.cumsum(_rng(seed_arrivals).exponential(1.0 / rate, size=total))
    i = np.arange(total)
    if switch_step is not None:
        fp32 = (i // nseq) < switch_step
    else:
        fp32 = _rng(seed_dtypes).random(total) < p32
    return t - t[0], i % nseq, i // nseq, fp32


def device_reflectors(torch, n, b, device, generator, dtype=None, complex_=False):
    """synthetic_reflectors drawn on the device with a torch generator (same
    structure and distribution, another random stream): for throughput runs
    and full-size tests whose inputs stand in for an upstream stage that
    produces them on the GPU.  Returns (hh, tau) 1-D device tensors (fp64,
    complex128 with complex_, unless dtype)."""
    _, _, _, LL = reflector_layout(n, b)
    N = LL.size
    L = torch.from_numpy(LL).to(device)
    pad = torch.arange(b, device=device)[None, :] >= L[:, None]
    if complex_:
        dt = dtype or torch.complex128
        h = np.sqrt(0.5) / np.sqrt(b)
        re = torch.randn((N, b), generator=generator, device=device, dtype=torch.float64) * h
        im = torch.randn((N, b), generator=generator, device=device, dtype=torch.float64) * h
        hh = torch.complex(re, im)
        del re, im
        hh[:, 0] = 1.0
        hh.masked_fill_(pad, 0.0)
        nrm2 = (hh.real * hh.real + hh.imag * hh.imag).sum(dim=1)
        th = torch.rand(N, generator=generator, device=device, dtype=torch.float64) * (2 * np.pi)
        tau = (1.0 - torch.polar(torch.ones_like(th), th)) / nrm2
        return hh.reshape(-1).to(dt), tau.to(dt)
    dt = dtype or torch.float64
    hh = torch.randn((N, b), generator=generator, device=device, dtype=torch.float64)
    hh *= 1.0 / np.sqrt(b)
    hh[:, 0] = 1.0
    hh.masked_fill_(pad, 0.0)
    tau = 2.0 / (hh * hh).sum(dim=1)
    tau.masked_fill_(L == 1, 0.0)
    return hh.reshape(-1).to(dt), tau.to(dt)


def device_block(torch, n, nev, device, generator, dtype=None, complex_=False):
    """gaussian_block drawn on the device: column-major (n, nev) tensor with
    N(0, 1/n) entries (complex: each part N(0, 1/(2n))); fp64 / complex128
    unless dtype."""
    if complex_:
        h = np.sqrt(0.5) / np.sqrt(n)
        re = torch.randn((nev, n), generator=generator, device=device, dtype=torch.float64) * h
        im = torch.randn((nev, n), generator=generator, device=device, dtype=torch.float64) * h
        z = torch.complex(re, im)
        del re, im
        return z.to(dtype or torch.complex128).t()
    z = torch.randn((nev, n), generator=generator, device=device, dtype=torch.float64)
    z *= 1.0 / np.sqrt(n)
    return z.to(dtype or torch.float64).t()


def synthetic_stage1(n, b, complex_=False, seed=0):
    """Random first-stage (full -> band) reflectors in the layout of the band
    -> full back-transformation: V (n x max(n-b, 1), column major) with
    column c holding v_c on rows c+b .. n-1 (unit lead at row c+b, entries
    of scale 1/sqrt(n-c-b) below, zeros above), tau (max(n-b, 1),) with
    tau = 2 / |v|^2 (real) or (1 - e^{i theta}) / |v|^2 (complex), so every
    H_c = I - tau v v^H is unitary.
    """
    N = max(n - b, 0)
    g = _rng(seed)
    dt = np.complex128 if complex_ else np.float64
    V = np.zeros((n, max(N, 1)), dtype=dt, order="F")
    tau = np.zeros(max(N, 1), dtype=dt)
    for c in range(N):
        L = n - c - b
        sc = 1.0 / np.sqrt(L)
        if complex_:
            h = np.sqrt(0.5) * sc
            v = g.standard_normal(L) * h + 1j * (g.standard_normal(L) * h)
        else:
            v = g.standard_normal(L) * sc
        v[0] = 1.0
        V[c + b:, c] = v
        nrm2 = float(np.sum(np.abs(v) ** 2))
        if complex_:
            tau[c] = (1.0 - np.exp(1j * g.uniform(0.0, 2.0 * np.pi))) / nrm2
        else:
            tau[c] = 2.0 / nrm2
    return V, tau
