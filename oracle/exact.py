"""Exact references on tiny periodic lattices.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Three independent ways to contract the same finite torus of Lx x Ly PEPS sites
(every site of the torus is one site of the unit cell, so the torus has
exactly Lx*Ly sites; Lx, Ly >= 2 so that no tensor meets itself):

* ``state_vector``      the wave function of Eq. PEPS as a dense vector, from
                        which <Psi|Psi> and any reduced density matrix follow;
* ``double_layer_rdm``  the reduced (double-layer) tensors of Eq. Tred on the
                        same torus;
* ``nested_rdm``        the nested single-layer network of Fig. NTN(c) on the
                        2Lx x 2Ly torus, with the Y tensors of the chosen sites
                        opened.

All three must agree to rounding.  This pins the nested construction
(network.py) and the impurity used for local operators.
"""
from __future__ import annotations

import torch

from .network import LT, as_t, bra_site, contract_all, cross_site, ket_site, phys_cross_open, phys_cross_site


def _peps_labels(x, y, Lx, Ly):
    return (f"h{(x - 1) % Lx},{y}", f"v{x},{(y - 1) % Ly}", f"h{x},{y}", f"v{x},{y}")


def state_vector(A, pattern):
    """Psi[s(0,0), s(1,0), ..., s(Lx-1,Ly-1)] of the PEPS on the Lx x Ly torus (row-major sites)."""
    A = as_t(A)
    Ly, Lx = len(pattern), len(pattern[0])
    assert Lx >= 2 and Ly >= 2
    ts = []
    for y in range(Ly):
        for x in range(Lx):
            ts.append(LT(A[pattern[y][x]], (f"s{x},{y}",) + _peps_labels(x, y, Lx, Ly)))
    psi = contract_all(ts)
    order = [f"s{x},{y}" for y in range(Ly) for x in range(Lx)]
    return psi.order(order)


def brute_rdm(A, pattern, sites):
    """rho[k_1..k_n, b_1..b_n] = sum_rest Psi[k, rest] Psi*[b, rest] for the listed PEPS sites."""
    psi = state_vector(A, pattern)
    Ly, Lx = len(pattern), len(pattern[0])
    flat = [(x, y) for y in range(Ly) for x in range(Lx)]
    keep = [flat.index(s) for s in sites]
    rest = [i for i in range(len(flat)) if i not in keep]
    p = psi.permute(keep + rest)
    dk = 1
    for i in keep:
        dk *= psi.shape[i]
    m = p.reshape(dk, -1)
    rho = m @ m.conj().T
    d = psi.shape[0]
    return rho.reshape([d] * (2 * len(sites)))


def double_layer_rdm(A, pattern, sites):
    """Same quantity from the reduced tensors T = sum_s A[s] A*[s] of Eq. Tred (open s at ``sites``)."""
    A = as_t(A)
    Ly, Lx = len(pattern), len(pattern[0])
    ts = []
    for y in range(Ly):
        for x in range(Lx):
            a = A[pattern[y][x]]
            l, u, r, dn = _peps_labels(x, y, Lx, Ly)
            ket = LT(a, (f"k{x},{y}", l + "k", u + "k", r + "k", dn + "k"))
            bra_labels = (f"b{x},{y}" if (x, y) in sites else f"k{x},{y}", l + "b", u + "b", r + "b", dn + "b")
            bra = LT(a.conj(), bra_labels)
            ts.append(ket * bra)            # the double-layer tensor of one site
    out = contract_all(ts)
    return out.order([f"k{x},{y}" for (x, y) in sites] + [f"b{x},{y}" for (x, y) in sites])


def nested_rdm(A, pattern, sites):
    """Same quantity from the nested single-layer network on the 2Lx x 2Ly torus."""
    A = as_t(A)
    d, D = A.shape[1], A.shape[2]
    Ly, Lx = len(pattern), len(pattern[0])
    NY, NX = 2 * Ly, 2 * Lx
    X, Y, Yo = cross_site(D), phys_cross_site(D, d), phys_cross_open(D, d)
    ts = []
    for I in range(NY):
        for J in range(NX):
            y, x = I // 2, J // 2
            labels = (f"H{I},{(J - 1) % NX}", f"V{(I - 1) % NY},{J}", f"H{I},{J}", f"V{I},{J}")
            kind = (I % 2, J % 2)
            a = A[pattern[y][x]]
            if kind == (0, 0):
                ts.append(LT(ket_site(a), labels))
            elif kind == (1, 1):
                ts.append(LT(bra_site(a), labels))
            elif kind == (1, 0):
                ts.append(LT(X, labels))
            elif (x, y) in sites:
                ts.append(LT(Yo, labels + (f"k{x},{y}", f"b{x},{y}")))
            else:
                ts.append(LT(Y, labels))
    out = contract_all(ts)
    return out.order([f"k{x},{y}" for (x, y) in sites] + [f"b{x},{y}" for (x, y) in sites])


def bond_expectation(rho2, h):
    """<h> = sum h[b_a b_b ; k_a k_b] rho[k_a k_b ; b_a b_b] / Tr rho for a two-site rho[k_a,k_b,b_a,b_b]."""
    d = rho2.shape[0]
    r = rho2.reshape(d * d, d * d)
    h = as_t(h)
    return (torch.einsum("ji,ij->", h, r) / torch.trace(r)).item()
