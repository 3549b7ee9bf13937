"""Seeded synthetic inputs for the GPP self-energy reduction.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic, so both the HIP path and the CPU oracle can use it.

Array names and index order follow the loop nest of Sec. II-A (pseudo-code of
the GPP kernel) and the array shapes named in Sec. III (v4, v7).  Fortran's
column-major ``X(ig, igp)`` becomes C row-major ``X[p][g]`` with ``g``
fastest:

* ``aqsmtemp``     complex128 ``[number_bands][ncouls]`` (only ``p < ngpown`` read)
* ``aqsntemp``     complex128 ``[number_bands][ncouls]``
* ``I_eps_array``  complex128 ``[ngpown][ncouls]``
* ``wtilde_array`` complex128 ``[ngpown][ncouls]``
* ``vcoul``        float64    ``[ncouls]``
* ``wx_array``     float64    ``[nfreq][number_bands]``

The paper's Si-214/Si-510 systems are real BerkeleyGW data that are not
available; the shapes and value ranges below are synthetic stand-ins.

Draw order with ``rng = numpy.random.default_rng(seed)`` (all uniforms are
``rng.uniform(lo, hi, shape)``):

1. band energies ``e_n`` ~ U[-1, 1) (number_bands)
2. ``e_lk`` ~ U[-1, 1) (scalar)
3. ``aqsmtemp`` real part, then imaginary part ~ U[-0.5, 0.5)
4. ``aqsntemp`` real, then imaginary ~ U[-0.5, 0.5)
5. ``I_eps_array`` real, then imaginary ~ U[-0.5, 0.5)
6. ``wtilde_array`` real ~ U[0.5, 2.0), then imaginary ~ U[-0.05, 0.05)
7. ``vcoul`` ~ U[0.1, 1.0)
8. ``wx_array[w][n] = e_lk - e_n + shift[w]`` with ``shift = (w - (nfreq-1)/2) / 2``
   (nfreq = 3 gives -0.5, 0, +0.5)
9. optional pole plant: ``k = round(fraction * ngpown * ncouls)`` distinct flat
   (p, g) indices via ``rng.choice(.., replace=False)``, then ``k`` flat (w, n)
   indices via ``rng.integers``, then ``delta_re``, ``delta_im`` ~ U[-1e-6, 1e-6);
   ``wtilde[p][g] = wx[w][n] + delta_re + 1j * delta_im``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

__all__ = [
    "Dims", "Problem", "Workload", "WORKLOADS", "make_problem",
    "make_problem_device", "make_upstream_grad", "make_fd_entries",
    "batched_dims", "small_batched_dims", "make_batched", "workload",
]


@dataclass(frozen=True)
class Dims:
    """Loop bounds of the GPP reduction (Sec. II-A): bands, occupied bands,
    G rows (ncouls), G' columns (ngpown) and output frequencies."""

    number_bands: int
    nvband: int
    ncouls: int
    ngpown: int
    nfreq: int

    def as_tuple(self):
        return (self.number_bands, self.nvband, self.ncouls, self.ngpown,
                self.nfreq)

    @property
    def ch_terms(self) -> int:
        return self.number_bands * self.ngpown * self.ncouls * self.nfreq

    @property
    def sx_terms(self) -> int:
        return self.nvband * self.ngpown * self.ncouls * self.nfreq


@dataclass
class Problem:
    dims: Dims
    aqsmtemp: np.ndarray
    aqsntemp: np.ndarray
    I_eps_array: np.ndarray
    wtilde_array: np.ndarray
    vcoul: np.ndarray
    wx_array: np.ndarray
    seed: object = None
    # energy of the quasiparticle state (e_lk) and the spacing of the nfreq
    # frequencies around it: wx_array[w][n] = e_lk + (w - (nfreq-1)/2) * freq_step - e_n
    e_lk: Optional[float] = None
    freq_step: float = 0.5

    def arrays(self):
        return (self.aqsmtemp, self.aqsntemp, self.I_eps_array,
                self.wtilde_array, self.vcoul, self.wx_array)


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: sizes, seed and pole-plant fraction."""

    name: str
    dims: Dims
    seed: int
    pole_fraction: float = 0.0


# Named after what they are.  The first is small enough for the oracle to
# finish in well under a second; the second has the per-task shape of the
# paper's Si-system run (bands/igp/ig magnitudes of Sec. II-A); the third is
# a larger system with planted near-poles; the fourth is the adjoint case.
WORKLOADS: Dict[str, Workload] = {
    "small": Workload("gpp-nb32-nv2-ng512-np64-nw3",
                      Dims(32, 2, 512, 64, 3), 0),
    "si": Workload("gpp-nb512-nv2-ng32768-np1638-nw3",
                   Dims(512, 2, 32768, 1638, 3), 1),
    "large": Workload("gpp-nb1024-nv4-ng65536-np3276-nw3-poles1pct",
                      Dims(1024, 4, 65536, 3276, 3), 2, 0.01),
    "adjoint": Workload("gpp-adjoint-nb256-nv2-ng16384-np819-nw3",
                        Dims(256, 2, 16384, 819, 3), 4),
}

BATCHED_SEED = 3
BATCHED_STATES = 64


def workload(key: str) -> Workload:
    return WORKLOADS[key]


def _complex_uniform(rng, shape, lo_re, hi_re, lo_im, hi_im):
    out = np.empty(shape, dtype=np.complex128)
    out.real = rng.uniform(lo_re, hi_re, shape)
    out.imag = rng.uniform(lo_im, hi_im, shape)
    return out


def make_problem(dims: Dims, seed, pole_fraction: float = 0.0) -> Problem:
    """Draw one problem in the documented order (module docstring)."""
    nb, nv, ng, npw, nw = dims.as_tuple()
    rng = np.random.default_rng(seed)
    e_n = rng.uniform(-1.0, 1.0, nb)
    e_lk = rng.uniform(-1.0, 1.0)
    aqsm = _complex_uniform(rng, (nb, ng), -0.5, 0.5, -0.5, 0.5)
    aqsn = _complex_uniform(rng, (nb, ng), -0.5, 0.5, -0.5, 0.5)
    ieps = _complex_uniform(rng, (npw, ng), -0.5, 0.5, -0.5, 0.5)
    wt = _complex_uniform(rng, (npw, ng), 0.5, 2.0, -0.05, 0.05)
    vcoul = rng.uniform(0.1, 1.0, ng)
    shift = (np.arange(nw, dtype=np.float64) - (nw - 1) / 2.0) * 0.5
    wx = np.ascontiguousarray((e_lk - e_n)[None, :] + shift[:, None])
    if pole_fraction > 0.0:
        k = int(round(pole_fraction * npw * ng))
        flat_pg = rng.choice(npw * ng, size=k, replace=False)
        flat_wn = rng.integers(0, nw * nb, size=k)
        d_re = rng.uniform(-1e-6, 1e-6, k)
        d_im = rng.uniform(-1e-6, 1e-6, k)
        wtf = wt.reshape(-1)
        wtf[flat_pg] = wx.reshape(-1)[flat_wn] + d_re + 1j * d_im
    return Problem(dims, aqsm, aqsn, ieps, wt, vcoul, wx, seed, e_lk=float(e_lk))


def make_upstream_grad(nfreq: int, rng) -> tuple:
    """Random complex unit-norm upstream gradient on (achtemp, asxtemp):
    2*nfreq complex standard normals (real parts drawn first), scaled to unit
    2-norm over all 2*nfreq entries."""
    re = rng.standard_normal(2 * nfreq)
    im = rng.standard_normal(2 * nfreq)
    z = re + 1j * im
    z = z / np.sqrt(np.sum(re * re + im * im))
    return np.ascontiguousarray(z[:nfreq]), np.ascontiguousarray(z[nfreq:])


def make_fd_entries(dims: Dims, rng, count: int = 1000) -> dict:
    """Distinct random entries per differentiable array, for finite-difference
    checks.  aqsmtemp entries come from the used block (columns < ngpown)."""
    nb, _, ng, npw, _ = dims.as_tuple()

    def pick(rows, cols):
        k = min(count, rows * cols)
        flat = rng.choice(rows * cols, size=k, replace=False)
        return np.stack([flat // cols, flat % cols], axis=1)

    return {
        "wtilde_array": pick(npw, ng),
        "I_eps_array": pick(npw, ng),
        "aqsntemp": pick(nb, ng),
        "aqsmtemp": pick(nb, npw),
    }


def batched_dims(seed: int = BATCHED_SEED, nstates: int = BATCHED_STATES,
                 nfreq: int = 3, bands=(64, 512), rows256=(16, 128)) -> List[Dims]:
    """Per-state sizes of a batched workload: number_bands uniform in
    {bands[0]..bands[1]}, ncouls = 256 * uniform{rows256[0]..rows256[1]},
    ngpown = ncouls // 20, nvband = 2.  The defaults are the 64-state
    workload: 64..512 bands, 4096..32768 rows."""
    rng = np.random.default_rng(seed)
    nb = rng.integers(bands[0], bands[1] + 1, nstates)
    ng = 256 * rng.integers(rows256[0], rows256[1] + 1, nstates)
    return [Dims(int(b), 2, int(g), int(g) // 20, nfreq) for b, g in zip(nb, ng)]


# Many small states (a small system's quasiparticle states): 256 states of
# 32..128 bands and 1024..4096 rows, sizes from default_rng(5).  Each one
# alone fills a fraction of the GPU for tens of microseconds.
SMALL_BATCHED_SEED = 5
SMALL_BATCHED_STATES = 256
SMALL_BATCHED_BANDS = (32, 128)
SMALL_BATCHED_ROWS256 = (4, 16)


def small_batched_dims(nfreq: int = 3) -> List[Dims]:
    return batched_dims(SMALL_BATCHED_SEED, SMALL_BATCHED_STATES, nfreq,
                        SMALL_BATCHED_BANDS, SMALL_BATCHED_ROWS256)


TINY_BATCHED_SEED = 31
TINY_BATCHED_STATES = 3000


def tiny_batched_dims(nfreq: int = 3) -> List[Dims]:
    """Sizes of a set of many tiny states (1-6 bands, 1-100 G rows, 1-5 G'
    columns, nvband min(2, bands)), drawn from default_rng(31)."""
    rng = np.random.default_rng(TINY_BATCHED_SEED)
    out = []
    for _ in range(TINY_BATCHED_STATES):
        nb = int(rng.integers(1, 7))
        ng = int(rng.integers(1, 101))
        out.append(Dims(nb, min(2, nb), ng, int(rng.integers(1, min(ng, 5) + 1)), nfreq))
    return out


def make_batched(seed: int = BATCHED_SEED, nstates: int = BATCHED_STATES,
                 nfreq: int = 3, states: Optional[Sequence[int]] = None):
    """Yield (index, Problem) per state; state s draws from default_rng([seed, s])."""
    dims = batched_dims(seed, nstates, nfreq)
    idx = range(nstates) if states is None else states
    for s in idx:
        yield s, make_problem(dims[s], [seed, s])


def make_problem_device(dims: Dims, seed: int, device="cuda:0") -> dict:
    """The same value distributions as make_problem, drawn directly on the
    device with torch's generator (for throughput runs whose size makes
    host-side generation the bottleneck; not bit-identical to
    make_problem, so never used where an oracle value is compared)."""
    import torch
    nb, nv, ng, npw, nw = dims.as_tuple()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = torch.float64

    def uni(shape, lo, hi):
        return torch.rand(shape, generator=gen, dtype=f64, device=device) * (hi - lo) + lo

    e_n = uni((nb,), -1.0, 1.0)
    e_lk = uni((1,), -1.0, 1.0)
    cu = lambda shape, lr, hr, li, hi: torch.complex(uni(shape, lr, hr), uni(shape, li, hi))
    out = {
        "aqsmtemp": cu((nb, ng), -0.5, 0.5, -0.5, 0.5),
        "aqsntemp": cu((nb, ng), -0.5, 0.5, -0.5, 0.5),
        "I_eps_array": cu((npw, ng), -0.5, 0.5, -0.5, 0.5),
        "wtilde_array": cu((npw, ng), 0.5, 2.0, -0.05, 0.05),
        "vcoul": uni((ng,), 0.1, 1.0),
    }
    shift = (torch.arange(nw, dtype=f64, device=device) - (nw - 1) / 2.0) * 0.5
    out["wx_array"] = ((e_lk - e_n)[None, :] + shift[:, None]).contiguous()
    return out
