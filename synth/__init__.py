"""Seeded synthetic workloads for the ETD2RKds hot path.

This module only *describes* problems: grid sizes, domains, diffusion and
advection coefficients, reaction-model constants, step size, step count and
the seeded initial data.  It holds none of the integrator's arithmetic (no
operators, no matrix functions, no time stepping), so both the CPU oracle and
the GPU harness can read their inputs from it without sharing any code of the
method.

Conventions
-----------
* A grid tensor of order d has shape ``(n_1, ..., n_d)`` and is stored with
  the first index fastest ("column-major"), which is the ``vec`` ordering of
  Sec. 2 of the paper.  In numpy that is ``order='F'``; the device buffers
  hold the same bytes.
* Grid nodes are node-centred: ``x_i = a + i*(b-a)/(n-1)``, ``i = 0..n-1``.
* Seeded noise is ``numpy.random.default_rng(seed).uniform(lo, hi, N)`` laid
  out column-major, drawn for U first and then for V.

Reaction models and their constant vectors (the same order is used by the
C ABI, ``include/adr.h``):

* ``schnakenberg``  params = (gamma, a, b):
  g^u = gamma*(a - u + u^2 v),  g^v = gamma*(b - u^2 v)        (Sec. 4.1, eq. (12))
* ``fhn``           params = (rho, eps, a1, a0):
  g^u = rho*(u - u^3 - v),      g^v = rho*eps*(u - a1*v - a0)  (Sec. 4.2-4.3, eqs. (13)-(14))
* ``brusselator``   params = (A, B):
  g^u = A - (B+1) u + u^2 v,    g^v = B u - u^2 v              (Sec. 4.6, eq. (17))
* ``dib``           params = (rho, a1u, a2u, a3u, a4u, a1v, a2v, a3v, a4v, a5v):
  the morpho-chemical DIB model of Sec. 4.4, eq. (15)

The formulas are listed here as documentation of the parameter order only;
each side implements them on its own.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

MODELS = ("schnakenberg", "fhn", "brusselator")


@dataclasses.dataclass(frozen=True)
class Workload:
    """One two-component ADR problem on a tensor-product grid."""

    name: str
    n: Tuple[int, ...]                       # grid points per direction, n[0] fastest
    domain: Tuple[Tuple[float, float], ...]  # [a_mu, b_mu] per direction
    diff: Tuple[float, float]                # (delta^u, delta^v)
    vel_u: Tuple[float, ...]                 # advection velocity per direction, u
    vel_v: Tuple[float, ...]                 # advection velocity per direction, v
    model: str
    params: Tuple[float, ...]
    tau: float
    steps: int
    # initial state: "noise" = base + U[lo, hi]; "sine_bruss" / "bump_schnak" are
    # the deterministic initial data of Secs. 4.6 and 4.5
    init: str = "noise"
    base: Tuple[float, float] = (0.0, 0.0)
    noise: Tuple[float, float] = (0.0, 0.0)

    @property
    def d(self) -> int:
        return len(self.n)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def nodes(n: int, a: float, b: float) -> np.ndarray:
    """Node-centred grid points x_i = a + i*(b-a)/(n-1)."""
    return a + (b - a) * np.arange(n, dtype=np.float64) / (n - 1)


def _noise_pair(N: int, lo: float, hi: float, seed: int):
    rng = np.random.default_rng(seed)
    xi = rng.uniform(lo, hi, size=N)
    eta = rng.uniform(lo, hi, size=N)
    return xi, eta


def initial_state(w: Workload, seed: int = 0):
    """Return (U0, V0) as float64 arrays of shape ``w.n`` in Fortran order."""
    N = w.N
    if w.init == "noise":
        xi, eta = _noise_pair(N, w.noise[0], w.noise[1], seed)
        u = w.base[0] + xi
        v = w.base[1] + eta
        U = np.asfortranarray(u.reshape(w.n, order="F"))
        V = np.asfortranarray(v.reshape(w.n, order="F"))
        return U, V
    grids = np.meshgrid(*[nodes(n, a, b) for n, (a, b) in zip(w.n, w.domain)],
                        indexing="ij")
    if w.init == "sine_bruss":
        # Sec. 4.6: u0 = 1 + prod_mu sin(2 pi x_mu),  v0 = 3
        s = np.ones(w.n)
        for x in grids:
            s = s * np.sin(2.0 * math.pi * x)
        U = 1.0 + s
        V = np.full(w.n, 3.0)
    elif w.init == "bump_schnak":
        # Sec. 4.5: u0 = a+b + 1e-5 exp(-100 |x - (1/3,1/2,1/3)|^2),  v0 = b/(a+b)^2
        _, a, b = w.params
        centre = (1.0 / 3.0, 0.5, 1.0 / 3.0)
        r2 = sum((x - c) ** 2 for x, c in zip(grids, centre))
        U = a + b + 1e-5 * np.exp(-100.0 * r2)
        V = np.full(w.n, b / (a + b) ** 2)
    else:
        raise ValueError(f"unknown initial data {w.init!r}")
    return np.asfortranarray(U), np.asfortranarray(V)


# --------------------------------------------------------------------------
# The benchmark workloads (synthetic stand-ins for the paper's experiments).
# --------------------------------------------------------------------------

def schnakenberg_2d(n: int = 64, steps: int = 100, tau: float = 1e-3) -> Workload:
    """2D Schnakenberg on [0,1]^2: u_t = Lap u + 200(0.1-u+u^2v), v_t = 10 Lap v + 200(0.9-u^2v).

    Stand-in for Sec. 4.1 (which uses delta^v=10 and rho=1000 at 150^2 with
    MATLAB-seeded noise); equilibrium (a+b, b/(a+b)^2) = (1.0, 0.9).
    """
    g, a, b = 200.0, 0.1, 0.9
    return Workload(
        name=f"schnakenberg2d_{n}", n=(n, n), domain=((0.0, 1.0),) * 2,
        diff=(1.0, 10.0), vel_u=(0.0, 0.0), vel_v=(0.0, 0.0),
        model="schnakenberg", params=(g, a, b), tau=tau, steps=steps,
        init="noise", base=(a + b, b / (a + b) ** 2), noise=(-0.01, 0.01))


def fhn_3d(n: int = 128, steps: int = 200, tau: float = 1e-3) -> Workload:
    """3D FitzHugh-Nagumo on [0,1]^3: u_t = Lap u + u-u^3-v, v_t = 4 Lap v + 0.1(u-2v).

    Stand-in for Sec. 4.3 (same reaction structure, its own constants);
    equilibrium (0, 0).
    """
    return Workload(
        name=f"fhn3d_{n}", n=(n, n, n), domain=((0.0, 1.0),) * 3,
        diff=(1.0, 4.0), vel_u=(0.0,) * 3, vel_v=(0.0,) * 3,
        model="fhn", params=(1.0, 0.1, 2.0, 0.0), tau=tau, steps=steps,
        init="noise", base=(0.0, 0.0), noise=(-0.1, 0.1))


def brusselator_3d(n: int = 256, steps: int = 100, tau: float = 5e-3) -> Workload:
    """3D advective Brusselator on [0,1]^3, alpha = 0.1*(1, 0.5, 0.25), A=1, B=3.

    D_u = 1e-3, D_v = 5e-3; stand-in for Sec. 4.6; equilibrium (A, B/A) = (1, 3).
    """
    alpha = (0.1, 0.05, 0.025)
    A, B = 1.0, 3.0
    return Workload(
        name=f"brusselator3d_{n}", n=(n, n, n), domain=((0.0, 1.0),) * 3,
        diff=(1e-3, 5e-3), vel_u=alpha, vel_v=alpha,
        model="brusselator", params=(A, B), tau=tau, steps=steps,
        init="noise", base=(A, B / A), noise=(-0.01, 0.01))


def paper_brusselator_3d(n: int = 64, steps: int = 100, T: float = 1.0) -> Workload:
    """The advective Brusselator experiment of Sec. 4.6 / Table 6 (deterministic data).

    delta^u = 0.01, delta^v = 0.02, alpha^u = alpha^v = 0.1 on every axis,
    a_1^u = B = 1, a_2^u = A = 2, u0 = 1 + sin sin sin, v0 = 3, T = 1.
    """
    return Workload(
        name=f"paper_brusselator3d_{n}", n=(n, n, n), domain=((0.0, 1.0),) * 3,
        diff=(0.01, 0.02), vel_u=(0.1,) * 3, vel_v=(0.1,) * 3,
        model="brusselator", params=(2.0, 1.0), tau=T / steps, steps=steps,
        init="sine_bruss")


def dib_a4v(a1v: float, a4u: float, a3v: float) -> float:
    """The constant a_4^v that Sec. 4.4 chooses so that (0, a_4^u) is an
    equilibrium of the DIB reaction (a Turing-unstable one)."""
    return a1v * (1.0 - a4u) * (1.0 - a3v + a3v * a4u) / (a4u * (1.0 + a3v * a4u))


def dib_2d(n: int = 200, steps: int = 1250, T: float = 2.5) -> Workload:
    """The 2D morpho-chemical DIB experiment of Sec. 4.4 / Table 4: [0,20]^2,
    delta^u = 1, delta^v = 20, rho = 25/4 and the constants printed there;
    initial data (0, a_4^u) plus 1e-5 * U(0, 1) noise (seeded here; the paper
    seeds MATLAB's generator, which this does not reproduce)."""
    a1u, a2u, a3u, a4u = 10.0, 1.0, 66.0, 0.5
    a1v, a2v, a3v, a5v = 3.0, 2.5, 0.2, 1.5
    a4v = dib_a4v(a1v, a4u, a3v)
    return Workload(
        name=f"dib2d_{n}", n=(n, n), domain=((0.0, 20.0),) * 2,
        diff=(1.0, 20.0), vel_u=(0.0, 0.0), vel_v=(0.0, 0.0),
        model="dib", params=(25.0 / 4.0, a1u, a2u, a3u, a4u, a1v, a2v, a3v, a4v, a5v),
        tau=T / steps, steps=steps, init="noise", base=(0.0, a4u), noise=(0.0, 1e-5))


def paper_schnakenberg_3d(n: int = 80, steps: int = 50, T: float = 0.4) -> Workload:
    """The advective Schnakenberg experiment of Sec. 4.5 / Table 5 (deterministic data)."""
    return Workload(
        name=f"paper_schnakenberg3d_{n}", n=(n, n, n), domain=((0.0, 1.0),) * 3,
        diff=(0.05, 1.0), vel_u=(0.01,) * 3, vel_v=(0.01,) * 3,
        model="schnakenberg", params=(100.0, 0.1305, 0.7695), tau=T / steps,
        steps=steps, init="bump_schnak")


def with_shape(w: Workload, n: Sequence[int]) -> Workload:
    """Same physics on another grid (velocities truncated/padded to the new d)."""
    n = tuple(int(x) for x in n)
    d = len(n)
    dom = tuple(w.domain[0] for _ in range(d))
    vu = tuple((list(w.vel_u) + [w.vel_u[-1]] * d)[:d])
    vv = tuple((list(w.vel_v) + [w.vel_v[-1]] * d)[:d])
    return w.replace(name=f"{w.model}_{'x'.join(map(str, n))}", n=n, domain=dom,
                     vel_u=vu, vel_v=vv)


# --------------------------------------------------------------------------
# Batched and serving workloads (grid sides, constants and arrivals drawn
# from a seed).
# --------------------------------------------------------------------------

BATCH_SIDES = (64, 96, 128, 192, 256, 384, 512)


def batched_schnakenberg_2d(count: int = 64, steps: int = 200, tau: float = 1e-3,
                            seed: int = 0):
    """Independent 2D Schnakenberg instances with seeded sides and constants."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        side = int(rng.choice(BATCH_SIDES))
        a = float(rng.uniform(0.05, 0.2))
        b = float(rng.uniform(0.7, 1.0))
        dv = float(rng.uniform(8.0, 12.0))
        g = float(rng.uniform(100.0, 400.0))
        out.append(Workload(
            name=f"batch{k}_schnak_{side}", n=(side, side), domain=((0.0, 1.0),) * 2,
            diff=(1.0, dv), vel_u=(0.0, 0.0), vel_v=(0.0, 0.0),
            model="schnakenberg", params=(g, a, b), tau=tau, steps=steps,
            init="noise", base=(a + b, b / (a + b) ** 2), noise=(-0.01, 0.01)))
    return out


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float          # seconds after stream start
    workload: Workload
    seed: int


def serving_stream(count: int = 64, rate: float = 20.0, seed: int = 0,
                   max_side_2d: int = 1024, max_side_3d: int = 192):
    """Poisson arrivals of mixed 2D/3D requests with seeded sizes and step counts."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    sides2 = [s for s in (128, 192, 256, 384, 512, 768, 1024) if s <= max_side_2d]
    sides3 = [s for s in (32, 48, 64, 96, 128, 160, 192) if s <= max_side_3d]
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        steps = int(rng.integers(50, 501))
        tau = float(np.exp(rng.uniform(np.log(1e-4), np.log(5e-3))))
        kind = rng.uniform()
        if kind < 0.5:
            w = with_shape(schnakenberg_2d(), (int(rng.choice(sides2)),) * 2)
        elif kind < 0.75:
            w = with_shape(fhn_3d(), (int(rng.choice(sides3)),) * 3)
        else:
            w = with_shape(brusselator_3d(), (int(rng.choice(sides3)),) * 3)
        w = w.replace(tau=tau, steps=steps, name=f"req{k}_{w.name}")
        reqs.append(Request(rid=k, arrival=t, workload=w, seed=int(rng.integers(1 << 30))))
    return reqs


CONFIGS = {
    "schnakenberg2d_64": schnakenberg_2d,
    "fhn3d_128": fhn_3d,
    "brusselator3d_256": brusselator_3d,
}
