"""Lattice geometry and index conventions (Sec. 3: on-site tensor legs p,l,u,r,d;
bonds pair r(x) with l(x+e_x) and u(x) with d(x+e_y)).

* Lx x Ly periodic lattice, site i(x) = x2*Lx + x1, V = Lx*Ly.
* link l = 2 i(x) + mu: mu = 0 joins x -> x+e1, mu = 1 joins x -> x+e2.
* Fock modes (brute force): mode 5 i + slot, slot p=0, l=1, u=2, r=3, d=4.
* virtual Majorana space (covariance form): n = 8V, index 8 i + 2 v + t with
  v = l 0, u 1, r 2, d 3 and t = 0, 1 the two Majoranas of the mode.
* the gauge field acts on the outgoing leg of each link (the "top and right"
  legs of Sec. 3.1): r(x) for mu = 0, u(x) for mu = 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SLOT_P, SLOT_L, SLOT_U, SLOT_R, SLOT_D = range(5)
VSLOT_L, VSLOT_U, VSLOT_R, VSLOT_D = range(4)


@dataclass(frozen=True)
class Lattice:
    Lx: int
    Ly: int

    @property
    def V(self) -> int:
        return self.Lx * self.Ly

    @property
    def n_links(self) -> int:
        return 2 * self.V

    @property
    def n(self) -> int:
        """Order of the virtual matrices M(G) and G = M^-1."""
        return 8 * self.V

    def site(self, x1: int, x2: int) -> int:
        return (x2 % self.Ly) * self.Lx + (x1 % self.Lx)

    def coords(self, i: int):
        return i % self.Lx, i // self.Lx

    def shift(self, i: int, d1: int, d2: int) -> int:
        x1, x2 = self.coords(i)
        return self.site(x1 + d1, x2 + d2)

    def link(self, i: int, mu: int) -> int:
        return 2 * i + mu

    def link_sites(self, ell: int):
        """(x, y): the link runs from site x (out end) to site y (in end)."""
        i, mu = divmod(ell, 2)
        j = self.shift(i, 1, 0) if mu == 0 else self.shift(i, 0, 1)
        return i, j

    def link_modes(self, ell: int):
        """Fock mode indices (out, in) of the two virtual modes the bond joins."""
        i, mu = divmod(ell, 2)
        _, j = self.link_sites(ell)
        if mu == 0:
            return 5 * i + SLOT_R, 5 * j + SLOT_L
        return 5 * i + SLOT_U, 5 * j + SLOT_D

    def link_majoranas(self, ell: int):
        """Virtual-space Majorana indices (out0, out1, in0, in1) of link ell."""
        i, mu = divmod(ell, 2)
        _, j = self.link_sites(ell)
        if mu == 0:
            o, q = 8 * i + 2 * VSLOT_R, 8 * j + 2 * VSLOT_L
        else:
            o, q = 8 * i + 2 * VSLOT_U, 8 * j + 2 * VSLOT_D
        return np.array([o, o + 1, q, q + 1])

    def plaquette_links(self, i: int):
        """Links (x,e1), (x+e1,e2), (x+e2,e1), (x,e2) of the plaquette at x."""
        return (self.link(i, 0), self.link(self.shift(i, 1, 0), 1),
                self.link(self.shift(i, 0, 1), 0), self.link(i, 1))

    def site_links(self, i: int):
        """The four links touching site i (two outgoing, two incoming)."""
        return (self.link(i, 0), self.link(i, 1),
                self.link(self.shift(i, -1, 0), 0), self.link(self.shift(i, 0, -1), 1))
