"""Counter-based random inputs (SplitMix64) and the base materials of the workload.

SplitMix64 is the generator published by Steele, Lea and Flood (OOPSLA 2014,
"Fast splittable pseudorandom number generators"): add the golden-ratio
increment 0x9E3779B97F4A7C15 to the state, then apply the two xor-shift-multiply
rounds (constants 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB) and a final
xor-shift.  Here it is used counter-style: the state is a pure function of
(seed, item, slot), so any item's numbers can be regenerated on their own.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB

# Layout of one parameter record (one macro Gauss point): 11 doubles.
PARAM_FIELDS = ("T_celsius", "c_wt", "t_years",
                "f_mE", "f_mnu", "f_mk", "f_mD",
                "f_yE", "f_ynu", "f_yk", "f_yD")

# Base constants of the synthetic plain-weave workload (matrix isotropic, yarn
# transversely isotropic; moduli in GPa, k in W/mK, D normalised).
BASE_MATERIALS = dict(
    E=3.5, nu=0.35, k=0.2, D=1.0,
    E1=55.0, E2=12.0, G12=4.5, nu12=0.28, nu23=0.4,
    k1=0.8, k2=0.3, D1=0.5, D2=0.2,
)


def _mix(z):
    """Output function of SplitMix64 applied to uint64 numpy arrays (wrapping)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def splitmix64(seed, item, slot):
    """64-bit output for counter (seed, item, slot); arrays broadcast.

    state = seed * 2^32 + item * 64 + slot (mod 2^64), then one SplitMix64 step.
    """
    seed = np.asarray(seed, dtype=np.uint64)
    item = np.asarray(item, dtype=np.uint64)
    slot = np.asarray(slot, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = (seed << np.uint64(32)) + item * np.uint64(64) + slot
        state = state + np.uint64(_GAMMA)
    return _mix(state)


def uniform01(seed, item, slot):
    """Double in [0, 1): top 53 bits of the SplitMix64 output times 2^-53."""
    z = splitmix64(seed, item, slot)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def draw_params(seed: int, n: int, first_item: int = 0,
                T_range=(20.0, 60.0), c_range=(0.0, 1.5), t_range=(0.0, 10.0),
                factor_spread=0.1) -> np.ndarray:
    """n parameter records [n, 11] for the degraded (batched) workload.

    Slots: 0 -> T ~ U(T_range) deg C, 1 -> c ~ U(c_range) wt%, 2 -> t ~ U(t_range)
    years, 3..10 -> the eight property factors ~ U(1-spread, 1+spread).
    """
    items = np.arange(first_item, first_item + n, dtype=np.uint64)[:, None]
    slots = np.arange(11, dtype=np.uint64)[None, :]
    u = uniform01(seed, items, slots)
    out = np.empty((n, 11), dtype=np.float64)
    out[:, 0] = T_range[0] + (T_range[1] - T_range[0]) * u[:, 0]
    out[:, 1] = c_range[0] + (c_range[1] - c_range[0]) * u[:, 1]
    out[:, 2] = t_range[0] + (t_range[1] - t_range[0]) * u[:, 2]
    out[:, 3:] = (1.0 - factor_spread) + 2.0 * factor_spread * u[:, 3:]
    return out


def draw_factors_only(seed: int, n: int, first_item: int = 0, factor_spread=0.1) -> np.ndarray:
    """Records with no exposure (T = 20 C, c = 0, t = 0) and seeded factors only.

    With c = 0 the degradation law leaves the matrix untouched, which is the
    undegraded single-RVE workload.
    """
    p = draw_params(seed, n, first_item, factor_spread=factor_spread)
    p[:, 0] = 20.0
    p[:, 1] = 0.0
    p[:, 2] = 0.0
    return p


def batch_sizes_c2(seed: int, n_rves: int, choices=(8, 12, 16, 20, 24)) -> np.ndarray:
    """Mesh size (cells per side) of each RVE in a mixed-size batch, uniform over choices."""
    u = uniform01(seed, np.arange(n_rves, dtype=np.uint64), np.uint64(63))
    idx = np.minimum((u * len(choices)).astype(np.int64), len(choices) - 1)
    return np.asarray(choices, dtype=np.int64)[idx]


def uniform_block(seed: int, stream: int, count: int) -> np.ndarray:
    """count doubles in [0, 1) of one stream: element e uses counter (seed, item=e, slot=stream).

    stream must be below 64 so that streams never share a counter.  Used for
    synthetic network weights and synthetic training rows in tests.
    """
    if not 0 <= stream < 64:
        raise ValueError("stream must be in [0, 64)")
    return uniform01(seed, np.arange(count, dtype=np.uint64), stream)
