"""Reverse-mode derivative of the CTMRG energy (Eq. AD).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The differentiated function is

    E(A) = energy after n sweeps started from a given environment env0,

with env0 held constant: the shortened chain of Sec. IV, where the paper
suggests taking the gradient from a supplied or nearly converged environment
instead of differentiating the whole iteration.  Starting from the fixed
sites-only environment instead makes E_n a chaotic function of A on random
tensors (a 1e-13 change of A reaches order one within a few sweeps), so its
derivative would carry no information; from a converged env0 the iteration is
contracting and E is smooth.

Every step is plain PyTorch (float64, CPU) and is differentiated by torch's
autograd, except the projector block (N, S) -> (P, Q) of Eqs. PQ/QRSVD.  Its
forward is the paper's QR + SVD; its derivative is written out here from the
equivalent form P = S^T V_rho Lambda~^(-1/2), Q = N^T U_rho Lambda~^(-1/2) with
rho = N S^T = (Q_n U) Lambda (Q_s V)^T, which needs no inverse of the
(often singular) R factors.  The SVD derivative is the textbook thin-SVD
formula with the Lorentzian-broadened F_ij = D_ij / (D_ij^2 + (eta m_ij)^2),
D_ij = s_j^2 - s_i^2, m_ij = max(s_i^2, s_j^2): only pairs whose squared
singular values agree to a relative eta are damped.  (A width fixed by s_1
alone would damp every pair of small kept singular values, which carry large
weights s^(-1/2) in P and Q, and bias the gradient.)
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from .ctmrg import check_cut, corner_spectra, projector_signs, sweep, truncated_inverse_sqrt
from .network import nested_cell, site_frames
from .rdm import energy_from_rdms, plaquette_rdm


def svd_backward(U, s, V, Ub, sb, Vb, eta, inv_mask):
    """A_bar for A = U diag(s) V^T (thin, real) given U_bar, s_bar, V_bar.

    ``inv_mask`` marks the columns whose U_bar / V_bar may be non-zero; 1/s is
    only formed there.
    """
    r = s.shape[0]
    s2 = s * s
    Dl = s2[None, :] - s2[:, None]                     # s_j^2 - s_i^2
    scale = torch.maximum(s2[None, :], s2[:, None])
    den = Dl * Dl + (eta * scale) ** 2
    # the broadened 1/D is D/(D^2 + width^2), which is 0 at D = 0 (also when
    # both singular values vanish and the width with them)
    F = torch.where(den > 0, Dl / torch.where(den > 0, den, torch.ones_like(den)), torch.zeros_like(den))
    F.fill_diagonal_(0.0)
    UtUb = U.T @ Ub
    VtVb = V.T @ Vb
    core = (F * (UtUb - UtUb.T)) * s[None, :] + torch.diag(sb) + s[:, None] * (F * (VtVb - VtVb.T))
    Ab = U @ core @ V.T
    sinv = torch.where(inv_mask, 1.0 / torch.where(inv_mask, s, torch.ones_like(s)), torch.zeros_like(s))
    Ab = Ab + ((Ub - U @ UtUb) * sinv[None, :]) @ V.T
    Ab = Ab + (U * sinv[None, :]) @ (Vb - V @ VtVb).T
    return Ab


class Projectors(torch.autograd.Function):
    """(N, S) -> (P, Q) of Eq. PQ with a hand-written derivative."""

    @staticmethod
    def forward(ctx, N, S, chi, cutoff, eta):
        Qn, Rn = torch.linalg.qr(N, mode="reduced")
        Qs, Rs = torch.linalg.qr(S, mode="reduced")
        M = Rn @ Rs.T
        U, s, Vh = torch.linalg.svd(M, full_matrices=False)
        check_cut(s, N, S)
        V = Vh.T
        k, w = truncated_inverse_sqrt(s, chi, cutoff)
        P = (Rs.T @ V[:, :k]) * w
        # gauge: the signs of the kept pairs (u_k, v_k) (another valid SVD)
        sg = projector_signs(P)
        U, V = U.clone(), V.clone()
        U[:, :k] *= sg
        V[:, :k] *= sg
        P = P * sg
        Q = (Rn.T @ U[:, :k]) * w
        ctx.save_for_backward(N, S, Qn @ U, Qs @ V, s, w)
        ctx.k, ctx.eta = k, eta
        return P, Q, s

    @staticmethod
    def backward(ctx, Pb, Qb, sb_unused):
        N, S, Ur, Vr, s, w = ctx.saved_tensors
        k, eta = ctx.k, ctx.eta
        X = Vr[:, :k] * w                  # P = S^T X
        Y = Ur[:, :k] * w                  # Q = N^T Y
        Sb = X @ Pb.T
        Nb = Y @ Qb.T
        Xb = S @ Pb
        Yb = N @ Qb
        r = s.shape[0]
        Ub = torch.zeros_like(Ur)
        Vb = torch.zeros_like(Vr)
        Vb[:, :k] = Xb * w
        Ub[:, :k] = Yb * w
        wb = (Vr[:, :k] * Xb).sum(0) + (Ur[:, :k] * Yb).sum(0)
        sb = torch.zeros_like(s)
        sb[:k] = wb * (-0.5) * w ** 3         # d(s^-1/2)/ds; zero where w = 0
        mask = torch.zeros(r, dtype=torch.bool)
        mask[:k] = w != 0
        rhob = svd_backward(Ur, s, Vr, Ub, sb, Vb, eta, mask)
        Nb = Nb + rhob @ S
        Sb = Sb + rhob.T @ N
        return Nb, Sb, None, None, None


def projector_fn(eta):
    def proj(N, S, chi, cutoff):
        return Projectors.apply(N, S, chi, cutoff, eta)
    return proj


def detach_env(env):
    return [[{k: v.detach().clone() for k, v in e.items()} for e in row] for row in env]


def energy_after_sweeps(A, pattern, chi, env0, n_sweeps, H, terms, cutoff=1e-10, eta=1e-12,
                        use_checkpoint=True):
    """E(A) after ``n_sweeps`` sweeps from the constant environment ``env0``; differentiable in A.

    Returns (E, env_final).  With ``use_checkpoint`` each sweep and each
    plaquette density matrix is recomputed during the backward pass instead of
    stored (torch.utils.checkpoint), which bounds memory to one sweep's or one
    plaquette's intermediates.
    """
    sites, _ = nested_cell(A, pattern)
    frames = site_frames(sites)
    proj = projector_fn(eta)
    env = env0
    keys = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")
    NY, NX = len(env), len(env[0])

    def one(A_, *flat):
        sites_ = site_frames(nested_cell(A_, pattern)[0])
        e = [[{k: flat[(I * NX + J) * 8 + n] for n, k in enumerate(keys)} for J in range(NX)] for I in range(NY)]
        e = sweep(sites_, e, chi, cutoff, proj=proj)
        return tuple(e[I][J][k] for I in range(NY) for J in range(NX) for k in keys)

    for _ in range(n_sweeps):
        flat = tuple(env[I][J][k] for I in range(NY) for J in range(NX) for k in keys)
        if use_checkpoint and A.requires_grad:
            out = checkpoint(one, A, *flat, use_reentrant=False)
        else:
            out = one(A, *flat)
        env = [[{k: out[(I * NX + J) * 8 + n] for n, k in enumerate(keys)} for J in range(NX)] for I in range(NY)]
    Ly, Lx = len(pattern), len(pattern[0])
    needed = sorted({(t[0], t[1]) for t in terms})
    flat = tuple(env[I][J][k] for I in range(NY) for J in range(NX) for k in keys)

    def rdm(px, py, A_, *flat_):
        e = [[{k: flat_[(I * NX + J) * 8 + n] for n, k in enumerate(keys)} for J in range(NX)] for I in range(NY)]
        return plaquette_rdm(nested_cell(A_, pattern)[0], e, px, py)

    rdms = {}
    for p in needed:
        if use_checkpoint and A.requires_grad:
            # recomputed in the backward pass: one plaquette's intermediates alive at a time
            rdms[p] = checkpoint(rdm, p[0], p[1], A, *flat, use_reentrant=False)
        else:
            rdms[p] = rdm(p[0], p[1], A, *flat)
    return energy_from_rdms(rdms, H, terms, Lx * Ly), env


def energy_and_grad(A, pattern, chi, env0, n_sweeps, H, terms, cutoff=1e-10, eta=1e-12, use_checkpoint=True):
    """(E, dE/dA, final environment) for ``energy_after_sweeps``."""
    A = torch.as_tensor(A, dtype=torch.float64).clone().requires_grad_(True)
    E, env = energy_after_sweeps(A, pattern, chi, detach_env(env0), n_sweeps, H, terms, cutoff, eta, use_checkpoint)
    (g,) = torch.autograd.grad(E, A)
    return E.item(), g, detach_env(env)


def fixed_point_grad(A, pattern, chi, env_star, H, terms, cutoff=1e-10, eta=1e-12, tol=1e-12, max_iter=500):
    """dE/dA of the converged energy E(A) = E(env*(A), A), where env* = f(env*, A) is the
    fixed point of the sweep map f (Eq. AD taken at the fixed point; Sec. IV).

    Implicit differentiation of env* = f(env*, A) gives
        dE/dA = dE/dA|_env + lam df/dA,   lam = dE/denv + lam df/denv,
    and lam = sum_k mu_k with mu_0 = dE/denv and mu_{k+1} = mu_k df/denv.  Each
    term is a vector-Jacobian product of one recorded sweep at (env*, A); the
    series stops once |mu_k| <= tol |mu_0| (it converges where the iteration
    itself is contracting).  The result is the limit n -> infinity of the
    gradient of ``energy_after_sweeps`` from env*.  env* must be a fixed point
    entry by entry (the gauge reading of ``ctmrg``).

    Returns (E, dE/dA, iterations, |f(env*) - env*|_max / |env*|_max).
    """
    A = torch.as_tensor(A, dtype=torch.float64).clone().requires_grad_(True)
    keys = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")
    NY, NX = len(env_star), len(env_star[0])
    leaves = [env_star[I][J][k].detach().clone().requires_grad_(True)
              for I in range(NY) for J in range(NX) for k in keys]
    env = [[{k: leaves[(I * NX + J) * 8 + n] for n, k in enumerate(keys)} for J in range(NX)] for I in range(NY)]
    frames = site_frames(nested_cell(A, pattern)[0])
    out = sweep(frames, env, chi, cutoff, proj=projector_fn(eta))
    outs = [out[I][J][k] for I in range(NY) for J in range(NX) for k in keys]
    gap = max((o.detach() - l.detach()).abs().max().item() for o, l in zip(outs, leaves)) / \
        max(l.detach().abs().max().item() for l in leaves)
    Ly, Lx = len(pattern), len(pattern[0])
    sites = nested_cell(A, pattern)[0]
    needed = sorted({(t[0], t[1]) for t in terms})
    rdms = {p: plaquette_rdm(sites, out, p[0], p[1]) for p in needed}
    E = energy_from_rdms(rdms, H, terms, Lx * Ly)
    # first term: dE/dA|_env + mu_0 df/dA (mu_0 = dE/d out) and mu_1 = mu_0 df/denv
    gs = torch.autograd.grad(E, [A] + leaves, retain_graph=True, allow_unused=True)
    grad = gs[0].clone()
    mu = [g if g is not None else torch.zeros_like(l) for g, l in zip(gs[1:], leaves)]
    norm0 = max(m.abs().max().item() for m in mu)
    it = 0
    while it < max_iter and norm0 > 0:
        it += 1
        gs = torch.autograd.grad(outs, [A] + leaves, grad_outputs=mu, retain_graph=True, allow_unused=True)
        grad += gs[0]
        mu = [g if g is not None else torch.zeros_like(l) for g, l in zip(gs[1:], leaves)]
        if max(m.abs().max().item() for m in mu) <= tol * norm0:
            break
    return E.item(), grad.detach(), it, gap
