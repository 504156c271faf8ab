"""Multi-site CTMRG on the nested cell (Sec. II C, Fig. CTMRG, Eqs. PQ and QRSVD).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Environment of nested position (I, J): four corners and four edges, each with
its legs listed in the order in which one meets them going counter-clockwise
around the site (this makes the labels invariant under quarter turns):

    C1[down, right]  top-left        T1[left, s, right]  above   (s = site up leg)
    C2[left, down]   top-right       T2[up, s, down]     right   (s = site right leg)
    C3[up, left]     bottom-right    T3[right, s, left]  below   (s = site down leg)
    C4[right, up]    bottom-left     T4[down, s, up]     left    (s = site left leg)

Turning the lattice a quarter turn counter-clockwise maps C2->C1, C3->C2,
C4->C3, C1->C4 and T2->T1, T3->T2, T4->T3, T1->T4 with unchanged arrays, so
the right, up and down moves are the left move in a turned frame (Sec. II C
treats them as the left move repeated in the other directions).

Readings of points the paper leaves open:
* start: by default every environment tensor is the neighbouring nested site
  with its outward legs summed against all-ones vectors; a caller may pass
  any starting environment instead (fine-tuned states such as products of
  singlets or decoupled chains need a generic one: from the all-ones start
  their projectors are exactly rank-deficient and the iteration stays in a
  wrong invariant sector);
* projectors keep chi' = min(chi, number of singular values of M); singular
  values below ``cutoff * s_1`` (default 1e-10) get a zero in place of
  s^(-1/2): smaller ones carry directions fixed only by rounding and, with
  weights s^(-1/2), make even weakly entangled states iterate chaotically;
* every updated tensor is divided by its Frobenius norm, and its sign is
  chosen so that its first entry within a relative 1e-9 (GAUGE_TIE) of the
  largest magnitude is positive;
* a sweep is the left, right, up and down moves in that order; the column
  steps of a move go in increasing order in the move's own frame;
* convergence: delta = max over all corners of the L1 distance between the
  normalised (sum 1) singular-value spectra of consecutive sweeps;
* gauge: the sign of every kept singular pair (u_k, v_k) of M, which flips
  column k of both P and Q, is chosen so that the first entry of P's column
  k within GAUGE_TIE of its largest magnitude is positive (ties that hold in
  exact arithmetic, as in every column of the double-layer network's
  projectors, are then decided the same way whatever the rounding): P does not
  depend on the sign conventions of the QR, so every implementation makes the
  same choice, and a converged environment is then a fixed point of the
  sweep entry by entry (which the fixed-point derivative needs);
* a cut whose bond density matrix rho = N S^T vanishes to working precision
  (largest singular value of M at most 1e-12 |N|_F |S|_F, where rounding
  alone leaves about 1e-16) carries no environment: Lambda~^(-1/2) of Eq. PQ
  is undefined there and the step raises ``DegenerateCut``.
"""
from __future__ import annotations

import torch

from .network import nested_cell, rotate_grid_ccw, site_frames

SLOT_ROT = {"C1": "C2", "C2": "C3", "C3": "C4", "C4": "C1",
            "T1": "T2", "T2": "T3", "T3": "T4", "T4": "T1"}


def rotate_env_ccw(env):
    """Environment seen in the frame turned a quarter turn counter-clockwise."""
    return rotate_grid_ccw(env, lambda e: {k: e[SLOT_ROT[k]] for k in SLOT_ROT})


def init_env(sites):
    """Starting environment: the nested neighbour with its outward legs summed (reading)."""
    NY, NX = len(sites), len(sites[0])
    env = [[None] * NX for _ in range(NY)]
    for I in range(NY):
        for J in range(NX):
            s = lambda di, dj: sites[(I + di) % NY][(J + dj) % NX]
            env[I][J] = {
                "C1": s(-1, -1).sum(dim=(0, 1)).permute(1, 0),     # [d, r]
                "T1": s(-1, 0).sum(dim=1).permute(0, 2, 1),        # [l, d, r]
                "C2": s(-1, 1).sum(dim=(1, 2)),                    # [l, d]
                "T2": s(0, 1).sum(dim=2).permute(1, 0, 2),         # [u, l, d]
                "C3": s(1, 1).sum(dim=(2, 3)).permute(1, 0),       # [u, l]
                "T3": s(1, 0).sum(dim=3).permute(2, 1, 0),         # [r, u, l]
                "C4": s(1, -1).sum(dim=(0, 3)).permute(1, 0),      # [r, u]
                "T4": s(0, -1).sum(dim=0).permute(2, 1, 0),        # [d, r, u]
            }
    return env


# relative size of the largest singular value of M below which a cut is empty
DEGENERATE_CUT = 1e-12


class DegenerateCut(ArithmeticError):
    """The bond density matrix of a cut is zero to working precision (no projector exists)."""


def check_cut(s, N, S):
    """Raise ``DegenerateCut`` if s_1 <= DEGENERATE_CUT * |N|_F |S|_F."""
    scale = (torch.linalg.norm(N.detach()) * torch.linalg.norm(S.detach())).item()
    if not s[0].item() > DEGENERATE_CUT * scale:
        raise DegenerateCut(f"cut carries no weight: s_1 = {s[0].item():.3e}, |N||S| = {scale:.3e}")


def truncated_inverse_sqrt(s, chi, cutoff):
    """Lambda~^(-1/2) of the chi' = min(chi, len(s)) largest singular values (pseudo-inverse)."""
    k = min(chi, s.shape[0])
    sk = s[:k]
    keep = sk > cutoff * s[0].detach()
    safe = torch.where(keep, sk, torch.ones_like(sk))
    return k, torch.where(keep, safe.rsqrt(), torch.zeros_like(sk))


# Relative width of a tie in the gauge rules: entries whose magnitudes are
# equal in exact arithmetic (the ket-bra exchange symmetry of a reduced tensor
# makes such pairs in every projector column of the double-layer network)
# differ by rounding only, so the sign is taken from the first entry within
# this width of the largest magnitude, which does not depend on where the
# rounding falls.
GAUGE_TIE = 1e-9


def _sign_entry(a):
    """Index (along dim 0) of the first entry of |a| within GAUGE_TIE of the column maximum."""
    m = a.max(dim=0).values
    return (a >= m * (1.0 - GAUGE_TIE)).to(torch.int8).argmax(dim=0)


def projector_signs(P):
    """+1/-1 per column: the sign of the column's first entry within a relative
    GAUGE_TIE of its largest magnitude (+1 for a zero column)."""
    idx = _sign_entry(P.detach().abs())
    v = P.detach()[idx, torch.arange(P.shape[1])]
    return torch.where(v < 0, -torch.ones_like(v), torch.ones_like(v))


def bond_projectors(N, S, chi, cutoff):
    """P, Q of Eq. PQ from the half systems N and S of Eq. QRSVD.

    N is [a1a2, a5a6] and S is [a3a4, a5a6].  N = Q_n R_n and S = Q_s R_s
    (reduced QR), R_n R_s^T = U Lambda V^T, and with Lambda~ the chi largest
    singular values P = R_s^T V Lambda~^(-1/2), Q = R_n^T U Lambda~^(-1/2);
    N P Q^T S^T is then the rank-chi truncated SVD of rho = N S^T.  Column
    signs as in ``projector_signs`` (the gauge reading of the module).
    """
    Rn = torch.linalg.qr(N, mode="reduced")[1]
    Rs = torch.linalg.qr(S, mode="reduced")[1]
    M = Rn @ Rs.T
    U, s, Vh = torch.linalg.svd(M, full_matrices=False)
    check_cut(s, N, S)
    k, w = truncated_inverse_sqrt(s, chi, cutoff)
    P = (Rs.T @ Vh[:k].T) * w
    Q = (Rn.T @ U[:, :k]) * w
    sg = projector_signs(P)
    return P * sg, Q * sg, s


def half_systems(sites, env, I, J):
    """N and S for the cut between rows I and I+1 at column step J (Fig. CTMRG c).

    Returns N[(h, z'), (e, z)] (rows: right cut of the upper half, columns:
    left cut) and S likewise for the lower half, plus the shapes of the left
    cut (chi leg, site leg) used to reshape the projectors.
    """
    NY, NX = len(sites), len(sites[0])
    I1, J1 = (I + 1) % NY, (J + 1) % NX
    e, s = env[I][J], sites[I][J]
    ul = torch.einsum("ab,bxc,eya,yxrz->crez", e["C1"], e["T1"], e["T4"], s)
    e, s = env[I][J1], sites[I][J1]
    ur = torch.einsum("cxf,fg,gyh,lxyz->clhz", e["T1"], e["C2"], e["T2"], s)
    e, s = env[I1][J], sites[I1][J]
    dl = torch.einsum("aye,ba,cwb,yxrw->excr", e["T4"], e["C4"], e["T3"], s)
    e, s = env[I1][J1], sites[I1][J1]
    dr = torch.einsum("hyg,gf,fwc,lxyw->hxcl", e["T2"], e["C3"], e["T3"], s)
    N = torch.einsum("crez,crhw->hwez", ul, ur)
    S = torch.einsum("excr,hwcr->hwex", dl, dr)
    nh, nw, ne, nz = N.shape
    sh, sw, se, sx = S.shape
    assert (ne, nz) == (se, sx)
    return N.reshape(nh * nw, ne * nz), S.reshape(sh * sw, se * sx), (ne, nz)


def normalized(t):
    """t / |t|_F with the sign that makes its first entry within a relative
    GAUGE_TIE of the largest magnitude positive."""
    flat = t.detach().reshape(-1)
    sg = -1.0 if flat[_sign_entry(flat.abs())] < 0 else 1.0
    return t * (sg / torch.linalg.norm(t))


def left_move(sites, env, chi, cutoff, proj=None, record=None):
    """One left move: for every column J, all projectors of the column, then all updates.

    Position (I, J+1) receives (Fig. CTMRG b)
        C1 <- [C1 T1](I,J) P_{I-1}
        T4 <- Q_{I-1}^T [T4 s](I,J) P_I
        C4 <- [C4 T3](I,J) Q_I
    each divided by its Frobenius norm; P_I attaches to the upper side of the
    cut between rows I and I+1, Q_I to the lower side.  ``proj`` may replace
    ``bond_projectors`` (the adjoint module passes one with a hand-written
    derivative).
    """
    proj = proj or bond_projectors
    NY, NX = len(sites), len(sites[0])
    env = [[dict(e) for e in row] for row in env]
    for J in range(NX):
        J1 = (J + 1) % NX
        P, Q = [None] * NY, [None] * NY
        for I in range(NY):
            N, S, (ne, nz) = half_systems(sites, env, I, J)
            p, q, sv = proj(N, S, chi, cutoff)
            P[I] = p.reshape(ne, nz, -1)
            Q[I] = q.reshape(ne, nz, -1)
            if record is not None:
                record.append(sv)
        new = []
        for I in range(NY):
            Im = (I - 1) % NY
            e, s = env[I][J], sites[I][J]
            C1 = torch.einsum("ab,bxc,axk->kc", e["C1"], e["T1"], P[Im])
            T4 = torch.einsum("eya,yxrz,axm,ezk->krm", e["T4"], s, Q[Im], P[I])
            C4 = torch.einsum("ba,cwb,awk->ck", e["C4"], e["T3"], Q[I])
            new.append((normalized(C1), normalized(T4), normalized(C4)))
        for I in range(NY):
            env[I][J1]["C1"], env[I][J1]["T4"], env[I][J1]["C4"] = new[I]
    return env


MOVE_FRAMES = (("left", 0), ("right", 2), ("up", 1), ("down", 3))


def sweep(frames, env, chi, cutoff, proj=None):
    """One CTMRG iteration: left, right, up and down moves (Sec. II C)."""
    frame = 0
    for _, f in MOVE_FRAMES:
        while frame != f:
            env = rotate_env_ccw(env)
            frame = (frame + 1) % 4
        env = left_move(frames[f], env, chi, cutoff, proj=proj)
    while frame != 0:
        env = rotate_env_ccw(env)
        frame = (frame + 1) % 4
    return env


def spectra_delta(new, old):
    """delta = max over corners of the L1 distance of two stacks of normalised spectra (rows = corners)."""
    return (new - old).abs().sum(dim=1).max().item()


def corner_spectra(env, chi):
    """Normalised singular values (sum 1, zero-padded to chi) of every corner, in a fixed order."""
    out = []
    for row in env:
        for e in row:
            for k in ("C1", "C2", "C3", "C4"):
                s = torch.linalg.svdvals(e[k].detach())
                s = s / s.sum()
                pad = torch.zeros(chi, dtype=s.dtype)
                n = min(chi, s.shape[0])
                pad[:n] = s[:n]
                out.append(pad)
    return torch.stack(out)


class CTM:
    """Oracle CTMRG state for one set of site tensors."""

    def __init__(self, A, pattern, chi, cutoff=1e-10, env0=None):
        """``env0``: optional starting environment in the flat layout of ``env_to_flat``;
        by default the sites-derived start of ``init_env`` is used."""
        self.pattern, self.chi, self.cutoff = pattern, chi, cutoff
        self.sites, self.kinds = nested_cell(A, pattern)
        self.frames = site_frames(self.sites)
        self.env = init_env(self.sites) if env0 is None else env_from_flat(env0, self.sites, chi)
        self.spectra = corner_spectra(self.env, chi)

    def run(self, max_sweeps, tol=0.0, proj=None):
        """Sweep until delta < tol or ``max_sweeps``; returns (sweeps done, last delta)."""
        delta = float("inf")
        n = 0
        for n in range(1, max_sweeps + 1):
            self.env = sweep(self.frames, self.env, self.chi, self.cutoff, proj=proj)
            sp = corner_spectra(self.env, self.chi)
            delta = spectra_delta(sp, self.spectra)
            self.spectra = sp
            if delta < tol:
                break
        return n, delta


ENV_SLOTS = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")
SITE_LEG = {"T1": 1, "T2": 2, "T3": 3, "T4": 0}      # which site leg (l,u,r,d) an edge touches


def env_slot_shapes(sites, chi):
    """Shapes of the chi-padded flat environment layout, position-major (I, J), then slot."""
    shapes = []
    for row in sites:
        for s in row:
            for k in ENV_SLOTS:
                shapes.append((chi, chi) if k[0] == "C" else (chi, s.shape[SITE_LEG[k]], chi))
    return shapes


def env_to_flat(env, sites, chi):
    """Zero-pad every chi leg to chi and concatenate (position-major, slots C1..C4, T1..T4)."""
    out = []
    for I, row in enumerate(sites):
        for J, _ in enumerate(row):
            for k in ENV_SLOTS:
                t = env[I][J][k].detach()
                if k[0] == "C":
                    p = torch.zeros(chi, chi, dtype=t.dtype)
                    p[: t.shape[0], : t.shape[1]] = t
                else:
                    p = torch.zeros(chi, t.shape[1], chi, dtype=t.dtype)
                    p[: t.shape[0], :, : t.shape[2]] = t
                out.append(p.reshape(-1))
    return torch.cat(out)


def env_from_flat(flat, sites, chi):
    """Inverse of ``env_to_flat`` (keeps the padded chi x ... x chi shapes)."""
    flat = torch.as_tensor(flat, dtype=torch.float64)
    env, off = [], 0
    shapes = iter(env_slot_shapes(sites, chi))
    for row in sites:
        erow = []
        for _ in row:
            e = {}
            for k in ENV_SLOTS:
                shp = next(shapes)
                n = 1
                for v in shp:
                    n *= v
                e[k] = flat[off: off + n].reshape(shp).clone()
                off += n
            erow.append(e)
        env.append(erow)
    assert off == flat.numel()
    return env
