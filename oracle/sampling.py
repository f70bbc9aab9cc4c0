"""Random draws of one Monte Carlo update, built on ``oracle.philox``.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings (the paper, Sec. II(c) step (c), only says the classical variable is
"randomly modified"):

* uniform in [0, 1):     u = (r >> 11) * 2**-53 for a 64-bit word r;
* uniform in [-1, 1):    v = (r >> 11) * 2**-52 - 1 (exact in FP64);
* proposed spin:         uniform on the unit sphere, independent of the
  current spin (a symmetric proposal, so the plain Metropolis ratio applies),
  by Marsaglia's method (Ann. Math. Stat. 43, 645 (1972)): draw (v1, v2)
  until s = v1^2 + v2^2 < 1 (s == 0 also rejected), then
  (2 v1 sqrt(1-s), 2 v2 sqrt(1-s), 1 - 2 s).  Each Philox block offers two
  pairs (words 0,1 then 2,3); block ``attempt`` a = 0, 1, ... is tried in turn.
  Only correctly rounded +, *, sqrt are used, evaluated one operation at a
  time in the order written, so any IEEE-754 implementation that does not
  contract them into fused multiply-adds reproduces the bits.
* counter layout:        (sweep, site, stream, attempt) with streams
  PROPOSAL=0, METROPOLIS=1 (word 0 -> u for the acceptance test, word 1 ->
  u1 for the first stage of delayed acceptance), SIZE=2 (word 0 -> cluster
  size class), INIT=3 (initial spins; sweep word = 2**64 - 1).

Pinned by: tests of the uniform moments of the sphere sampler, norm == 1,
and bitwise agreement with ``numpy.random.Philox``-driven re-derivation.
"""
import math

from .philox import philox4x64, MASK64

STREAM_PROPOSAL = 0
STREAM_METROPOLIS = 1
STREAM_SIZE = 2
STREAM_INIT = 3
INIT_SWEEP = MASK64
MAX_ATTEMPTS = 64

_TWO_M53 = 2.0 ** -53
_TWO_M52 = 2.0 ** -52


def u53(r: int) -> float:
    """Uniform double in [0, 1) from the top 53 bits of a 64-bit word."""
    return float(r >> 11) * _TWO_M53


def v52(r: int) -> float:
    """Uniform double in [-1, 1) from the top 53 bits of a 64-bit word."""
    return float(r >> 11) * _TWO_M52 - 1.0


def _marsaglia(v1: float, v2: float):
    s = v1 * v1
    s = s + v2 * v2
    if s >= 1.0 or s == 0.0:
        return None
    q = math.sqrt(1.0 - s)
    return ((2.0 * v1) * q, (2.0 * v2) * q, 1.0 - 2.0 * s)


def sphere_point(seed: int, sweep: int, site: int, stream: int):
    """Uniform point on S^2 for counter (sweep, site, stream, attempt)."""
    for attempt in range(MAX_ATTEMPTS):
        r = philox4x64((seed, 0), (sweep, site, stream, attempt))
        for a, b in ((r[0], r[1]), (r[2], r[3])):
            p = _marsaglia(v52(a), v52(b))
            if p is not None:
                return p
    raise RuntimeError("sphere sampler exhausted its attempts")


def proposal(seed: int, sweep: int, site: int):
    """Proposed new spin of ``site`` in ``sweep``."""
    return sphere_point(seed, sweep, site, STREAM_PROPOSAL)


def initial_spin(seed: int, site: int):
    """Isotropic random initial spin of ``site``."""
    return sphere_point(seed, INIT_SWEEP, site, STREAM_INIT)


def metropolis_uniforms(seed: int, sweep: int, site: int):
    """(u, u1): acceptance uniform and first-stage uniform of one update."""
    r = philox4x64((seed, 0), (sweep, site, STREAM_METROPOLIS, 0))
    return u53(r[0]), u53(r[1])


def size_class(seed: int, sweep: int, site: int, n_classes: int) -> int:
    """Index in [0, n_classes) of the cluster size used for this update:
    floor(hi32(r0) * n_classes / 2**32), exact integer arithmetic."""
    r = philox4x64((seed, 0), (sweep, site, STREAM_SIZE, 0))
    return ((r[0] >> 32) * n_classes) >> 32
