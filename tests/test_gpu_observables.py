"""Order parameters (Eqs. Mag1, Mag2) of the GPU library, through the C ABI,
against the CPU oracle: on the library's own density matrices (the kernel's
arithmetic alone) and on the oracle's density matrices from the same
environment (the whole chain)."""
import pytest
import torch

import synth
from oracle.ctmrg import CTM as OCTM
from oracle.observables import N_OBS, magnetization, plaquette_observables, plaquette_order
from oracle.rdm import plaquette_rdm as orho

pytestmark = pytest.mark.gpu

H = synth.heisenberg_bond()

CASES = [
    ("heis_1x1_D2", 1, 2, 8, [[0]], "uniform", 0),
    ("cell_2x2_D2", 4, 2, 8, [[0, 1], [2, 3]], "uniform", 1),
    ("cell_2x1_D3", 2, 3, 12, [[0, 1]], "normal", 2),
]


@pytest.fixture(scope="module")
def ctm_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_14414_amd as m
    return m


@pytest.mark.parametrize("name,nt,D,chi,pattern,dist,seed", CASES)
def test_observables_match_oracle(ctm_mod, name, nt, D, chi, pattern, dist, seed):
    print(f"[observables] {name} D={D} chi={chi}", flush=True)
    A = synth.site_tensors(nt, 2, D, seed, dist)
    Ly, Lx = len(pattern), len(pattern[0])
    env0 = synth.random_env_flat(chi, D, 2, Lx, Ly, seed + 10)
    g = ctm_mod.CTM(A, pattern, chi)
    g.set_env(torch.tensor(env0))
    assert g.observables().shape == (0, N_OBS)      # no energy call yet: no plaquettes
    terms = synth.heisenberg_terms(Lx, Ly)
    g.energy(H, terms)
    rhos = g.last_rdms()
    obs = g.observables()
    assert obs.shape == (rhos.shape[0], N_OBS)
    # the kernel's arithmetic on the same matrices
    for i in range(rhos.shape[0]):
        ref = plaquette_observables(rhos[i])
        assert torch.allclose(obs[i], ref, rtol=0, atol=1e-12), (i, (obs[i] - ref).abs().max())
    # the whole chain against the oracle's density matrices from the same environment
    o = OCTM(A, pattern, chi, env0=env0)
    plaqs = []
    for t in terms:
        if (t[0], t[1]) not in plaqs:
            plaqs.append((t[0], t[1]))
    ref_all = torch.stack([plaquette_observables(orho(o.sites, o.env, px, py)) for px, py in plaqs])
    assert torch.allclose(obs, ref_all, rtol=0, atol=1e-10)
    assert obs[:, 1:12:3].abs().max().item() == 0.0        # <S^y> of real tensors
    # composed order parameters agree as well
    Mg = magnetization(obs[:, :12].reshape(-1, 3))
    Mo = magnetization(ref_all[:, :12].reshape(-1, 3))
    assert abs(Mg.item() - Mo.item()) < 1e-10
    if obs.shape[0] > 1:
        assert abs(plaquette_order(obs[0], obs[1]).item() - plaquette_order(ref_all[0], ref_all[1]).item()) < 1e-10
    # a capacity below the count returns the leading plaquettes
    part = g.observables(capacity=1)
    assert part.shape == (1, N_OBS) and torch.equal(part[0], obs[0])
