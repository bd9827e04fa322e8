"""Velocity sets of the oracle (test infrastructure, see oracle/__init__.py).

The paper writes every scheme for a generic velocity set with weights w_q and
lattice sound speed c_s (Sec. 2.1.1, text after Eq. (35)); it spells out only
D1Q3 (Appendix A, Eq. (A.1)) and calls it the projection of the
higher-dimensional sets on one axis.  D2Q9 and D3Q19 below are the standard
isotropic sets with c_s^2 = 1/3.  Order of the directions is the oracle's own
and unrelated to the GPU code.
"""
from dataclasses import dataclass

import numpy as np

CS2 = 1.0 / 3.0


@dataclass(frozen=True)
class Lattice:
    name: str
    D: int
    v: np.ndarray      # (Q, D) integer velocities, component order (x, y, z)
    w: np.ndarray      # (Q,) weights
    opp: np.ndarray    # (Q,) index of -v_q

    @property
    def Q(self):
        return self.v.shape[0]


def _make(name, vel, wts):
    v = np.asarray(vel, dtype=np.int64).reshape(len(vel), -1)
    w = np.asarray(wts, dtype=np.float64)
    opp = np.array([next(j for j in range(len(v)) if np.all(v[j] == -v[i]))
                    for i in range(len(v))], dtype=np.int64)
    assert np.all(v[0] == 0), "q = 0 must be the rest velocity (delta_q of Eq. (39))"
    return Lattice(name, v.shape[1], v, w, opp)


def d1q3():
    # Appendix A, Eq. (A.1): velocities {0, 1, -1}; weights read off Eq. (A.2)
    return _make("D1Q3", [[0], [1], [-1]], [2 / 3, 1 / 6, 1 / 6])


def d2q9():
    vel = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
           (1, 1), (-1, 1), (-1, -1), (1, -1)]
    wts = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    return _make("D2Q9", vel, wts)


def d3q19():
    vel = [(0, 0, 0),
           (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
           (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
           (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
           (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    wts = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return _make("D3Q19", vel, wts)


def by_name(name):
    return {"D1Q3": d1q3, "D2Q9": d2q9, "D3Q19": d3q19}[name]()
