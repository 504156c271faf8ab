"""Nested single-layer network (Sec. II B, Eq. XY, Fig. NTN, footnote on bond dims).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The norm <Psi|Psi> of an iPEPS is rewritten as one square-lattice network in
which the ket tensor A and the bra tensor A* sit on different sites of a cell
twice as large in each direction.  For PEPS site (x, y) the nested sites are

    (2y,   2x)   K  = A   with its physical index fused into the right leg
    (2y,   2x+1) Y  = delta(l_k, r_k) delta(u_b, d_b) delta(s, s')   (Eq. XY)
    (2y+1, 2x)   X  = delta(l_b, r_b) delta(u_k, d_k)                (Eq. XY)
    (2y+1, 2x+1) B  = A*  with its physical index fused into the up leg

so ket bonds cross bra bonds at X and Y, and the physical index runs
K -> Y -> B.  Every nested tensor is stored with legs (l, u, r, d).  The left
and down legs of Y, the right leg of K and the up leg of B have dimension D*d
(the footnote to Sec. II C); all others have dimension D.  A fused leg is
(virtual index major, physical index minor).

Reading taken here (the figure is not available): the nested sites are
arranged [[K, Y], [X, B]] with the physical line routed K -> Y -> B.  The
exact torus checks in the tests confirm that this arrangement reproduces
<Psi|Psi> and <Psi|h|Psi>.
"""
from __future__ import annotations

import torch

DT = torch.float64


def as_t(x):
    return torch.as_tensor(x, dtype=DT)


def ket_site(A):
    """K[l, u, (r,s), d] = A[s, l, u, r, d]."""
    d, D = A.shape[0], A.shape[1]
    return A.permute(1, 2, 3, 0, 4).reshape(D, D, D * d, D)


def bra_site(A):
    """B[l, (u,s), r, d] = conj(A)[s, l, u, r, d]  (real tensors: conj is the identity)."""
    d, D = A.shape[0], A.shape[1]
    return A.conj().permute(1, 2, 0, 3, 4).reshape(D, D * d, D, D)


def cross_site(D):
    """X[l, u, r, d] = delta(l, r) delta(u, d)."""
    e = torch.eye(D, dtype=DT)
    return torch.einsum("lr,ud->lurd", e, e)


def phys_cross_site(D, d):
    """Y[(l,s), u, r, (d,s')] = delta(l, r) delta(u, d) delta(s, s')."""
    e, es = torch.eye(D, dtype=DT), torch.eye(d, dtype=DT)
    y = torch.einsum("lr,ud,st->lsurdt", e, e, es)
    return y.reshape(D * d, D, D, D * d)


def phys_cross_open(D, d):
    """Y with its physical line cut: Yo[(l,s), u, r, (d,s'), k, b] = delta(l,r) delta(u,d) delta(s,k) delta(s',b).

    ``k`` is the open ket index (coming from K) and ``b`` the open bra index
    (going to B); contracting k with b gives back Y.  This is the impurity
    used for local observables (Sec. II B).
    """
    e, es = torch.eye(D, dtype=DT), torch.eye(d, dtype=DT)
    y = torch.einsum("lr,ud,sk,tb->lsurdtkb", e, e, es, es)
    return y.reshape(D * d, D, D, D * d, d, d)


def nested_cell(A, pattern):
    """Nested sites of the unit cell, as a list of rows of (l,u,r,d) tensors.

    ``A`` has shape (n_tensors, d, D, D, D, D); ``pattern[y][x]`` picks the
    tensor at PEPS site (x, y).  Returns a 2*Ly by 2*Lx nested list and a
    parallel list of kinds ('K', 'Y', 'X', 'B').
    """
    A = as_t(A)
    d, D = A.shape[1], A.shape[2]
    Ly, Lx = len(pattern), len(pattern[0])
    X, Y = cross_site(D), phys_cross_site(D, d)
    sites = [[None] * (2 * Lx) for _ in range(2 * Ly)]
    kinds = [[None] * (2 * Lx) for _ in range(2 * Ly)]
    for y in range(Ly):
        for x in range(Lx):
            a = A[pattern[y][x]]
            sites[2 * y][2 * x], kinds[2 * y][2 * x] = ket_site(a), "K"
            sites[2 * y][2 * x + 1], kinds[2 * y][2 * x + 1] = Y, "Y"
            sites[2 * y + 1][2 * x], kinds[2 * y + 1][2 * x] = X, "X"
            sites[2 * y + 1][2 * x + 1], kinds[2 * y + 1][2 * x + 1] = bra_site(a), "B"
    return sites, kinds


def rotate_site_ccw(s):
    """Site seen after turning the lattice 90 degrees counter-clockwise.

    Up becomes left, right becomes up, down becomes right, left becomes down:
    new (l, u, r, d) = old (u, r, d, l).
    """
    return s.permute(1, 2, 3, 0)


def rotate_grid_ccw(grid, fn=lambda v: v):
    """Rotate a rows-by-cols nested list 90 degrees counter-clockwise.

    Old (I, J) in an NY x NX grid goes to (NX-1-J, I) in an NX x NY grid.
    """
    NY, NX = len(grid), len(grid[0])
    out = [[None] * NY for _ in range(NX)]
    for I in range(NY):
        for J in range(NX):
            out[NX - 1 - J][I] = fn(grid[I][J])
    return out


def site_frames(sites):
    """The nested cell in the four orientations used by the four moves.

    Frame f is the lattice turned f quarter turns counter-clockwise; a left
    move in frame 0, 2, 1, 3 is the left, right, up, down move of the
    original lattice.
    """
    frames = [sites]
    for _ in range(3):
        frames.append(rotate_grid_ccw(frames[-1], rotate_site_ccw))
    return frames


# --- labelled tensors for the exact / reference contractions ----------------

class LT:
    """A tensor whose axes carry string labels; shared labels are summed."""

    __slots__ = ("t", "labels")

    def __init__(self, t, labels):
        labels = tuple(labels)
        assert t.dim() == len(labels), (t.shape, labels)
        assert len(set(labels)) == len(labels), labels
        self.t, self.labels = t, labels

    def __mul__(self, other):
        return contract(self, other)

    def order(self, labels):
        labels = tuple(labels)
        assert sorted(labels) == sorted(self.labels), (labels, self.labels)
        return self.t.permute([self.labels.index(l) for l in labels])


def contract(a: LT, b: LT) -> LT:
    common = [l for l in a.labels if l in b.labels]
    ia = [a.labels.index(l) for l in common]
    ib = [b.labels.index(l) for l in common]
    for l in common:
        assert a.t.shape[a.labels.index(l)] == b.t.shape[b.labels.index(l)], l
    t = torch.tensordot(a.t, b.t, dims=(ia, ib))
    labels = [l for l in a.labels if l not in common] + [l for l in b.labels if l not in common]
    return LT(t, labels)


def contract_all(tensors):
    out = tensors[0]
    for t in tensors[1:]:
        out = contract(out, t)
    return out
