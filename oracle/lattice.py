"""D2Q9 and D3Q19 velocity sets (paper Section 2: "the D3Q19 or D2Q9 lattice model").

The paper names the two lattices but prints no table, no ordering and no value of the
lattice temperature T.  Readings used here:

* T = 1/3: the only value for which the standard weights satisfy
  sum_i w_i c_i c_i = T I (checked by the test-suite, not assumed).
* Ordering: index 0 is the rest velocity; the moving velocities come in opposite
  pairs (2k-1, 2k), so the opposite of i is i+1 for odd i and i-1 for even i.
  D2Q9:  +x, -x, +y, -y, (+x+y), (-x-y), (+x-y), (-x+y).
  D3Q19: +x, -x, +y, -y, +z, -z, (+x+y), (-x-y), (+x-y), (-x+y),
         (+x+z), (-x-z), (+x-z), (-x+z), (+y+z), (-y-z), (+y-z), (-y+z).

Velocities are stored as 3-vectors (x, y, z); D2Q9 has a zero z component.
"""
import numpy as np

T = 1.0 / 3.0


class Lattice:
    def __init__(self, name, c, w):
        self.name = name
        self.c = np.asarray(c, dtype=np.int64)          # (Q, 3)
        self.w = np.asarray(w, dtype=np.float64)        # (Q,)
        self.Q = len(self.w)
        self.D = 2 if name == "D2Q9" else 3
        self.opp = np.array([0] + [i + 1 if i % 2 == 1 else i - 1
                                   for i in range(1, self.Q)], dtype=np.int64)


def _d2q9():
    c = [(0, 0, 0),
         (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)]
    w = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4
    return Lattice("D2Q9", c, w)


def _d3q19():
    c = [(0, 0, 0),
         (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    w = [1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12
    return Lattice("D3Q19", c, w)


D2Q9 = _d2q9()
D3Q19 = _d3q19()


def lattice(q):
    """Lattice by velocity count (9 or 19)."""
    if q == 9:
        return D2Q9
    if q == 19:
        return D3Q19
    raise ValueError("lattice must be 9 or 19")
