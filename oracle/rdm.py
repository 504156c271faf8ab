"""2x2 reduced density matrix and energy (Eq. ExpH, impurity tensors of Sec. II B).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For the PEPS plaquette whose upper-left site is (x, y), the nested block is
rows 2y..2y+3 and columns 2x..2x+3 of the nested cell.  It is surrounded by
the multi-site environment of its border positions: C1 of the top-left
position, T1 of the four top positions, C2 of the top-right one, T2 of the four
right positions, C3, T3 of the bottom positions, C4 and T4 of the left
positions.  The four Y tensors of the block are opened (their physical line is
cut), which leaves rho[k_TL, k_TR, k_BL, k_BR ; b_TL, b_TR, b_BL, b_BR] with the
ket index k on the K side and the bra index b on the B side.

The raw rho is used, not a symmetrised one: the nested environment treats bra
and ket separately and need not be Hermitian (Sec. IV).

Contraction order (the network and its sum are fixed; only the order of the
pairwise contractions is chosen, for memory): each corner quadrant -- one
corner, its two pairs of edges and its 2x2 block of nested sites -- is
contracted first, then the upper two and the lower two quadrants, then the
two halves.  The largest intermediate is a half of chi^2 D^4 d^4 entries.
"""
from __future__ import annotations

import torch

from .network import LT, contract, contract_all

OPEN = {(0, 1): "TL", (0, 3): "TR", (2, 1): "BL", (2, 3): "BR"}
ORDER = ("TL", "TR", "BL", "BR")


def _ket_open_cross(D, d):
    """Y with the physical line cut, keeping the ket end: Yk[(l,s), u, r, d', k] = delta(l,r) delta(u,d') delta(s,k).

    Its down leg has dimension D only; the bra end of the cut line is exposed
    on the B tensor below (see ``_bra_open``).  Contracting Yk with that B over
    d' and k = b gives back Y followed by B.
    """
    e, es = torch.eye(D, dtype=torch.float64), torch.eye(d, dtype=torch.float64)
    return torch.einsum("lr,ud,sk->lsurdk", e, e, es).reshape(D * d, D, D, D, d)


def _bra_open(B, D, d):
    """B[l, (u,s'), r, d] with its fused up leg split: Bb[l, u, s', r, d]."""
    return B.reshape(B.shape[0], D, d, B.shape[2], B.shape[3])


def _block_tensors(sites, env, x, y):
    NY, NX = len(sites), len(sites[0])
    I0, J0 = 2 * y, 2 * x
    pos = lambda r, c: ((I0 + r) % NY, (J0 + c) % NX)
    E = lambda r, c: env[pos(r, c)[0]][pos(r, c)[1]]
    env_t = {
        "C1": LT(E(0, 0)["C1"], ("lB", "tA")),
        "C2": LT(E(0, 3)["C2"], ("tB", "rA")),
        "C3": LT(E(3, 3)["C3"], ("rB", "bA")),
        "C4": LT(E(3, 0)["C4"], ("bB", "lA")),
    }
    top = ["tA", "t0", "t1", "t2", "tB"]
    right = ["rA", "r0", "r1", "r2", "rB"]
    bottom = ["bB", "b0", "b1", "b2", "bA"]     # left to right
    left = ["lB", "l0", "l1", "l2", "lA"]       # top to bottom
    for c in range(4):
        env_t[f"T1{c}"] = LT(E(0, c)["T1"], (top[c], f"vT{c}", top[c + 1]))
        env_t[f"T3{c}"] = LT(E(3, c)["T3"], (bottom[c + 1], f"vB{c}", bottom[c]))
    for r in range(4):
        env_t[f"T2{r}"] = LT(E(r, 3)["T2"], (right[r], f"h{r}R", right[r + 1]))
        env_t[f"T4{r}"] = LT(E(r, 0)["T4"], (left[r + 1], f"h{r}L", left[r]))
    site_t = {}
    for r in range(4):
        for c in range(4):
            l = f"h{r}L" if c == 0 else f"h{r}{c - 1}"
            u = f"vT{c}" if r == 0 else f"v{r - 1}{c}"
            rt = f"h{r}R" if c == 3 else f"h{r}{c}"
            dn = f"vB{c}" if r == 3 else f"v{r}{c}"
            s = sites[pos(r, c)[0]][pos(r, c)[1]]
            if (r, c) in OPEN:                      # Y of a plaquette site: keep the ket end
                D = s.shape[1]
                d = s.shape[0] // D
                site_t[(r, c)] = LT(_ket_open_cross(D, d), (l, u, rt, dn, "k" + OPEN[(r, c)]))
            elif (r - 1, c) in OPEN:                # B below it: expose the bra end
                D = s.shape[0]
                d = s.shape[1] // D
                site_t[(r, c)] = LT(_bra_open(s, D, d), (l, u, "b" + OPEN[(r - 1, c)], rt, dn))
            else:
                site_t[(r, c)] = LT(s, (l, u, rt, dn))
    return env_t, site_t


def plaquette_rdm(sites, env, x, y):
    """rho as a (d^4 x d^4) matrix [(k_TL k_TR k_BL k_BR), (b_TL b_TR b_BL b_BR)], not normalised."""
    et, st = _block_tensors(sites, env, x, y)
    # each list starts at the corner and takes one edge and the site it touches at a time
    tl = contract_all([et["C1"], et["T10"], et["T40"], st[(0, 0)], et["T11"], st[(0, 1)], et["T41"], st[(1, 0)],
                       st[(1, 1)]])
    tr = contract_all([et["C2"], et["T13"], et["T20"], st[(0, 3)], et["T12"], st[(0, 2)], et["T21"], st[(1, 3)],
                       st[(1, 2)]])
    bl = contract_all([et["C4"], et["T43"], et["T30"], st[(3, 0)], et["T42"], st[(2, 0)], et["T31"], st[(3, 1)],
                       st[(2, 1)]])
    br = contract_all([et["C3"], et["T33"], et["T23"], st[(3, 3)], et["T32"], st[(3, 2)], et["T22"], st[(2, 3)],
                       st[(2, 2)]])
    rho = contract(contract(tl, tr), contract(bl, br))
    t = rho.order([f"k{n}" for n in ORDER] + [f"b{n}" for n in ORDER])
    d = t.shape[0]
    return t.reshape(d ** 4, d ** 4)


def pair_rdm(rho, a, b):
    """Two-site rho[(k_a k_b), (b_a b_b)] from the plaquette rho by tracing the other two sites."""
    d = round(rho.shape[0] ** 0.25)
    t = rho.reshape([d] * 8)
    letters_k = list("abcd")
    letters_b = list("efgh")
    others = [i for i in range(4) if i not in (a, b)]
    for i in others:
        letters_b[i] = letters_k[i]
    spec = "".join(letters_k) + "".join(letters_b) + "->" + letters_k[a] + letters_k[b] + letters_b[a] + letters_b[b]
    return torch.einsum(spec, t).reshape(d * d, d * d)


def energy_from_rdms(rdms, H, terms, n_sites):
    """E per site = (1/n_sites) sum coef * Tr(h rho_ab)/Tr(rho), <h> = sum h[b;k] rho[k;b] (Eq. ExpH)."""
    H = torch.as_tensor(H, dtype=torch.float64)
    E = 0.0
    for (px, py, a, b, coef) in terms:
        rho = rdms[(px, py)]
        r2 = pair_rdm(rho, a, b)
        E = E + coef * torch.einsum("ji,ij->", H, r2) / torch.trace(rho)
    return E / n_sites


def energy(ctm, H, terms):
    """Energy per site of a converged oracle CTM state for a list of plaquette terms."""
    Ly, Lx = len(ctm.pattern), len(ctm.pattern[0])
    needed = sorted({(t[0], t[1]) for t in terms})
    rdms = {p: plaquette_rdm(ctm.sites, ctm.env, p[0], p[1]) for p in needed}
    return energy_from_rdms(rdms, H, terms, Lx * Ly)


def normalized_plaquette_rdms(sites, env, Lx, Ly):
    """rho_p / Tr rho_p of every plaquette p = (x, y) of the Lx x Ly cell, in row-major order (y, then x)."""
    out = []
    for y in range(Ly):
        for x in range(Lx):
            r = plaquette_rdm(sites, env, x, y)
            out.append(r / torch.trace(r))
    return out


def rdm_delta(new, old):
    """Largest change of any entry of the normalised plaquette density matrices
    between two environments: a convergence measure that sees only what the
    energy and the order parameters are made of."""
    return max((a - b).abs().max().item() for a, b in zip(new, old))
