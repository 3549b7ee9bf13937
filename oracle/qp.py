"""Quasiparticle quantities from the self-energy at a few frequencies --
TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

The paper abstracts the GPP kernel from the Sigma module of BerkeleyGW
(Sec. II-A): the kernel's outputs achtemp[w] and asxtemp[w] are the
Coulomb-hole and screened-exchange sums of the self-energy at nfreq
frequencies E_w.  The step that consumes them is the linearised
quasiparticle equation; the paper does not print it, so the following is
the reading used on both sides (the library's epilogue and this oracle):

* the frequencies are equally spaced around the state's energy E:
  E_w = E + (w - m) h with m = (nfreq - 1) / 2 (nfreq odd, at least 3), the
  layout of the workloads' wx_array = E_w - e_n;
* Sigma(E_w) = achtemp[w] - asxtemp[w]: the screened exchange enters with a
  minus sign, since asxtemp is the unsigned exchange sum;
* dSigma/dE at E by the central difference over the two neighbours,
  (Sigma(E_{m+1}) - Sigma(E_{m-1})) / (2 h);
* the renormalisation Z = 1 / (1 - Re dSigma/dE), and the linearised
  quasiparticle energy E_qp = E + Z (Re Sigma(E) - V_xc) for a given
  exchange-correlation expectation value V_xc.

Plain Python complex arithmetic in fp64, step by step.
"""
from __future__ import annotations

import math

__all__ = ["quasiparticle"]


def quasiparticle(achtemp, asxtemp, freq_step, energy=0.0, vxc=0.0):
    """Sigma(E), dSigma/dE, Z and E_qp at the middle of nfreq equally spaced
    frequencies (module docstring).  achtemp, asxtemp: sequences of nfreq
    complex values.  Returns a dict with complex 'sigma' and 'dsigma', real
    'z' and 'e_qp', and 'sigma_all' (Sigma at every frequency)."""
    nw = len(achtemp)
    if len(asxtemp) != nw:
        raise ValueError("achtemp and asxtemp differ in length")
    if nw < 3 or nw % 2 == 0:
        raise ValueError(f"nfreq={nw}: need an odd number of frequencies, at least 3")
    if not (math.isfinite(freq_step) and freq_step > 0.0):
        raise ValueError("freq_step must be finite and positive")
    sigma_all = [complex(achtemp[w]) - complex(asxtemp[w]) for w in range(nw)]
    m = (nw - 1) // 2
    dsigma = (sigma_all[m + 1] - sigma_all[m - 1]) / (2.0 * freq_step)
    z = 1.0 / (1.0 - dsigma.real)
    e_qp = energy + z * (sigma_all[m].real - vxc)
    return {"sigma": sigma_all[m], "dsigma": dsigma, "z": z, "e_qp": e_qp,
            "sigma_all": sigma_all}
