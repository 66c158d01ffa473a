"""Flat-surface emission tables (the method's physics input).

The method samples the number, energy and direction of secondaries from
relations pre-computed for an ideally flat surface (section 2.2).  A table
set holds:

* ``yld``: secondary yield on a grid of primary energy E (log-uniform from
  ``E_min`` to ``E_max``, ``n_E`` points) by local incidence angle
  (uniform from 0 to 90 degrees, ``n_theta`` points), float32 [n_E, n_theta];
* ``cdf_E``/``cdf_F``: the secondary-energy CDF as points (E_k, F_k) with
  E_0 = 0, F_0 = 0, F nondecreasing and F_last = 1; the spectrum is the
  piecewise-linear CDF through these points;
* ``Ec``: the emission cut-off energy E_c = work function + Fermi energy
  (section 2.2); rays at or below it do not emit on a hit.

Kinds built here:

* ``vaughan``: a Vaughan-type yield curve with an exp(0.5 (1 - cos theta))
  angular factor and Chung-Everhart secondary energies (work function 4.5 eV);
* ``paper_w``: the tungsten yield fit of Eq. (seey), evaluated with the
  angle in degrees and the energy in eV (clipped at 0), with the same
  Chung-Everhart spectrum;
* ``constant``: a constant yield (verification special cases).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Tables:
    yld: np.ndarray  # float32 [n_E, n_theta]
    E_min: float
    E_max: float
    cdf_E: np.ndarray  # float32 [n_cdf]
    cdf_F: np.ndarray  # float32 [n_cdf]
    Ec: float = 10.0
    meta: dict = field(default_factory=dict)
    esee: np.ndarray | None = None  # float32 [n_E, n_theta]: E_SEE for the paper's emission rule
    emission: int = 0  # 0: energies from the CDF, cosine law; 1: the paper's one/two-daughter rule

    @property
    def n_E(self) -> int:
        return int(self.yld.shape[0])

    @property
    def n_theta(self) -> int:
        return int(self.yld.shape[1])

    def E_axis(self) -> np.ndarray:
        return np.exp(np.linspace(np.log(self.E_min), np.log(self.E_max), self.n_E))

    def theta_axis(self) -> np.ndarray:
        return np.linspace(0.0, 90.0, self.n_theta)


# ---------------------------------------------------------------- closed forms

def vaughan_yield(E, theta_deg, dmax=1.4, Emax=650.0):
    """Vaughan-type curve with zero threshold and exp(0.5 (1 - cos theta))."""
    E = np.asarray(E, dtype=np.float64)
    w = E / Emax
    k = np.where(w <= 1.0, 0.62, 0.25)
    with np.errstate(divide="ignore", invalid="ignore"):
        base = np.where(w > 0, (w * np.exp(1.0 - w)) ** k, 0.0)
    return dmax * base * np.exp(0.5 * (1.0 - np.cos(np.deg2rad(theta_deg))))


def paper_w_yield(E, alpha_deg):
    """Eq. (seey): flat-tungsten yield fit, alpha in degrees, E in eV."""
    E = np.asarray(E, dtype=np.float64)
    a = np.asarray(alpha_deg, dtype=np.float64)
    g = (3.05 + 1.7949e-5 * a * a + 6.15e-7 * E * E
         - (371.317 - np.exp(0.04826 * a)) / (87.602 + E)
         - 1.974e-3 * E - 0.1097 * np.cos(0.1201 + 2.469 * a))
    return g


def paper_w_esee(E, alpha_deg):
    """Secondary energy fit E_SEE(E, alpha) of section 2.2 (flat tungsten), in eV;
    alpha in degrees (the fit's sin(E) takes E as printed)."""
    E = np.asarray(E, dtype=np.float64)
    a = np.asarray(alpha_deg, dtype=np.float64)
    return 0.195 * E + 1.6e-4 * E * E + 0.148 * a * np.sin(E) + 3.44e-15 * E * a ** 7 - 6.54


def ce_cdf(E, phi=4.5):
    """Chung-Everhart CDF for density proportional to E / (E + phi)^4."""
    s = phi / (np.asarray(E, dtype=np.float64) + phi)
    return 1.0 - 3.0 * s * s + 2.0 * s ** 3


def ce_inverse(xi, phi=4.5):
    """Closed-form inverse of ce_cdf (root of 2 s^3 - 3 s^2 + 1 - xi = 0 in (0, 1])."""
    xi = np.asarray(xi, dtype=np.float64)
    s = 0.5 + np.cos((np.arccos(2.0 * xi - 1.0) + 4.0 * np.pi) / 3.0)
    with np.errstate(divide="ignore"):
        return phi * (1.0 / s - 1.0)


# ---------------------------------------------------------------- builders

def _ce_table(n_cdf: int, E_top: float, phi: float):
    E = np.empty(n_cdf, dtype=np.float64)
    E[0] = 0.0
    E[1:] = np.exp(np.linspace(np.log(1e-2), np.log(E_top), n_cdf - 1))
    F = ce_cdf(E, phi) / ce_cdf(E_top, phi)
    F[0] = 0.0
    F[-1] = 1.0
    F32 = np.maximum.accumulate(F.astype(np.float32))
    return E.astype(np.float32), F32


def make_tables(kind: str = "vaughan", n_E: int = 128, n_theta: int = 46, E_min: float = 1.0,
                E_max: float = 1.0e4, n_cdf: int = 512, phi: float = 4.5, Ec: float = 10.0,
                const: float = 1.0, dmax: float = 1.4, Emax: float = 650.0, emission: str | None = None,
                esee_const: float | None = None) -> Tables:
    """Flat-surface tables.  kind 'paper_w' is the paper's own tungsten fits
    (Eq. seey and E_SEE) with the paper's emission rule; emission='paper'
    selects that rule for any kind (E_SEE from the fit, or esee_const)."""
    Eax = np.exp(np.linspace(np.log(E_min), np.log(E_max), n_E))
    tax = np.linspace(0.0, 90.0, n_theta)
    if kind == "vaughan":
        y = vaughan_yield(Eax[:, None], tax[None, :], dmax=dmax, Emax=Emax)
    elif kind == "paper_w":
        y = np.clip(paper_w_yield(Eax[:, None], tax[None, :]), 0.0, 6.99)
        emission = "paper" if emission is None else emission
    elif kind == "constant":
        y = np.full((n_E, n_theta), const)
    else:
        raise ValueError(kind)
    cE, cF = _ce_table(n_cdf, E_max, phi)
    esee = None
    if emission == "paper":
        es = (np.full((n_E, n_theta), esee_const) if esee_const is not None
              else paper_w_esee(Eax[:, None], tax[None, :]))
        esee = np.ascontiguousarray(es, dtype=np.float32)
    elif emission not in (None, "spectrum"):
        raise ValueError(emission)
    return Tables(yld=np.ascontiguousarray(y, dtype=np.float32), E_min=E_min, E_max=E_max,
                  cdf_E=cE, cdf_F=cF, Ec=Ec,
                  meta=dict(kind=kind, phi=phi, const=const, dmax=dmax, Emax=Emax),
                  esee=esee, emission=1 if emission == "paper" else 0)


def bilinear_reference(t: Tables, E, alpha_deg):
    """Table value at (E, alpha): bilinear in (ln E, alpha), clamped at the edges.

    This is the documented interpolation rule of the table format, written
    with numpy for tests.
    """
    E = np.asarray(E, dtype=np.float64)
    a = np.asarray(alpha_deg, dtype=np.float64)
    x = (np.log(E) - np.log(t.E_min)) / (np.log(t.E_max) - np.log(t.E_min)) * (t.n_E - 1)
    x = np.clip(x, 0.0, t.n_E - 1)
    i = np.minimum(np.floor(x).astype(np.int64), t.n_E - 2)
    fx = x - i
    y = np.clip(a / 90.0 * (t.n_theta - 1), 0.0, t.n_theta - 1)
    j = np.minimum(np.floor(y).astype(np.int64), t.n_theta - 2)
    fy = y - j
    Y = t.yld.astype(np.float64)
    return ((1 - fx) * (1 - fy) * Y[i, j] + fx * (1 - fy) * Y[i + 1, j]
            + (1 - fx) * fy * Y[i, j + 1] + fx * fy * Y[i + 1, j + 1])
