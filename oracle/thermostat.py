"""FP64 oracle: the Andersen thermostat and its counter-based random numbers.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper couples its crystallisation run to an Andersen thermostat
(Sec. 5.2, the structure analysis results) without stating the collision rate or
how the random numbers are drawn.  Readings taken here (the device library
implements the same definitions independently):

* Collisions: after the second half kick of step s, each particle collides
  with probability p = nu * dt (nu: collision rate per unit time; nu * dt
  <= 1) and then takes a velocity drawn from the Maxwell-Boltzmann
  distribution at temperature T: each component sqrt(T / m) * N(0, 1)
  (k_B = 1 in reduced units).  The thermo sample of step s is taken before
  its collisions.
* Random numbers: Philox4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw,
  SC'11), key (seed, 0), counter (s, id, c, 0) for the global step s, the
  particle's id and block c.  A 64-bit output b gives the uniform
  U = (b >> 11) * 2^-53 in [0, 1).  Block 0 = (b0, b1, b2, b3): the particle
  collides iff U(b0) < p; then, with block 1 = (b4, ...),
      n1 = sqrt(-2 ln(1 - U(b1))) cos(2 pi U(b2))
      n2 = sqrt(-2 ln(1 - U(b1))) sin(2 pi U(b2))
      n3 = sqrt(-2 ln(1 - U(b3))) cos(2 pi U(b4))      (Box-Muller)
  so every draw depends only on (seed, s, id), not on how the particles
  are stored.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = (1 << 64) - 1
# Philox4x64 multipliers and Weyl key increments (the published constants)
_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block: four 64-bit words from a 4-word counter and
    a 2-word key (plain Python integers).  Each round multiplies words 0
    and 2 by the two constants (128-bit products), mixes the high halves
    with words 1 and 3 and the key, and the key advances by the Weyl
    increments between rounds."""
    x0, x1, x2, x3 = (int(c) & _M64 for c in ctr)
    k0, k1 = (int(k) & _M64 for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _M64
            k1 = (k1 + _W1) & _M64
        p0 = _M0 * x0
        p1 = _M1 * x2
        x0, x1, x2, x3 = (p1 >> 64) ^ x1 ^ k0, p1 & _M64, (p0 >> 64) ^ x3 ^ k1, p0 & _M64
    return x0, x1, x2, x3


def uniform53(b: int) -> float:
    """[0, 1) from the top 53 bits of a 64-bit word."""
    return (b >> 11) * (1.0 / 9007199254740992.0)


def andersen_draw(seed: int, step: int, pid: int, p: float):
    """(collides, (n1, n2, n3)) for particle pid at global step `step`."""
    b0, b1, b2, b3 = philox4x64_10((step, pid, 0, 0), (seed, 0))
    if not uniform53(b0) < p:
        return False, None
    b4 = philox4x64_10((step, pid, 1, 0), (seed, 0))[0]
    r1 = math.sqrt(-2.0 * math.log(1.0 - uniform53(b1)))
    t1 = 2.0 * math.pi * uniform53(b2)
    r2 = math.sqrt(-2.0 * math.log(1.0 - uniform53(b3)))
    t2 = 2.0 * math.pi * uniform53(b4)
    return True, (r1 * math.cos(t1), r1 * math.sin(t1), r2 * math.cos(t2))


def andersen(vel, ids, step: int, temperature: float, nu: float, dt: float, seed: int, mass: float = 1.0):
    """The collisions of step `step` applied to velocities (N, 3), returning
    the new velocities and the number of collisions."""
    v = np.array(vel, dtype=np.float64, copy=True)
    p = nu * dt
    sd = math.sqrt(temperature / mass)
    hits = 0
    for row, pid in enumerate(np.asarray(ids)):
        hit, n = andersen_draw(seed, step, int(pid), p)
        if hit:
            v[row] = (sd * n[0], sd * n[1], sd * n[2])
            hits += 1
    return v, hits
