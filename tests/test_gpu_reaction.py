"""GPU parity of the reaction step (Eq. 9-12 with the alpha-QSS integration
of Eq. 27-28) and of its splitting with the flow step, against the CPU
oracle, through the C ABI.

Workloads: the seeded synthetic mechanism (mass-balanced exchanges and
dissociations among the nine shock-bubble species, rate constants of
10^2..10^4 SI units at 1500 K) on random states at 1500 K, where it is stiff
(p dt up to ~20 per step of 1e-6 s), and a three-species dissociation.  Bar:
per field, max |U_gpu - U_oracle| <= 1e-12 max |U_f|; at full size (the
nine-species shock-bubble at 256^3, where the cold gas barely reacts) the
oracle integrates sampled cells one by one, and the partial densities are
judged against the largest density (most species start absent).
"""
import numpy as np
import pytest

import oracle as O
from conftest import oracle_objects
from paper_2403_05910_amd import workloads as W
from test_gpu_parity import field_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
R = O.xf_reaction
TOL = 1e-12


def _xf():
    from paper_2403_05910_amd import xf
    return xf


def _omech(mt):
    return R.Mechanism(mt.nu_f, mt.nu_b, mt.A, mt.B, mt.E, mt.third, mt.eff, mt.reversible, mt.s0)


def reacting_case(name):
    if name == "n9_1500K":
        tab = W.with_formation_enthalpies(W.sampled_table(W.W9, 0), 1)
        case = W.random_smooth_state(tab, (12, 10, 8), seed=3, T0=1500.0, bc=(1, 1, 0, 0, 0, 0))
        return case, W.synthetic_mechanism(W.W9, tab, 0, 12)
    if name == "n9_1500K_all_reactions":
        tab = W.with_formation_enthalpies(W.sampled_table(W.W9, 0), 2)
        case = W.random_smooth_state(tab, (9, 7, 6), seed=5, T0=1800.0)
        return case, W.synthetic_mechanism(W.W9, tab, 1, 32)
    tab = W.with_formation_enthalpies(W.sampled_table([2.0, 1.0, 28.0], 4), 3)
    case = W.random_smooth_state(tab, (20, 9, 1), seed=6, T0=2500.0)
    return case, W.synthetic_mechanism([2.0, 1.0, 28.0], tab, 2, 4)


def higher_order_case():
    """four species of molar masses 1, 2, 3 and 4 g/mol and reactions with
    two and three molecules of one species on a side: 3 A = C, 2 B = D (with
    a third body), A + C = D and 2 A + B = D, all reversible; rate constants
    of 10^2..10^4 SI units at 2000 K and entropy constants chosen as in the
    synthetic mechanism (S/R - h/(R T) within +-2 at 2000 K)"""
    Wg = [1.0, 2.0, 3.0, 4.0]
    tab = W.with_formation_enthalpies(W.sampled_table(Wg, 5), 4)
    case = W.random_smooth_state(tab, (11, 9, 7), seed=8, T0=2000.0)
    nu_f = np.array([[3, 0, 0, 0], [0, 2, 0, 0], [1, 0, 1, 0], [2, 1, 0, 0]])
    nu_b = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [0, 0, 0, 1], [0, 0, 0, 1]])
    rng = np.random.default_rng(9)
    nr, ns, T_ref = 4, 4, 2000.0
    k_ref = 10.0 ** rng.uniform(2.0, 4.0, nr)
    B = rng.uniform(-1.0, 1.5, nr)
    E = rng.uniform(0.0, 1.5e5, nr)
    A = k_ref / (T_ref ** B * np.exp(-E / (W.R_UNIVERSAL * T_ref)))
    third = np.array([False, True, False, False])
    eff = rng.uniform(0.5, 3.0, (nr, ns))
    a = np.asarray(tab.a)
    T = T_ref
    s_var = a[:, 0] * np.log(T) + a[:, 1] * T + a[:, 2] * T ** 2 / 2 + a[:, 3] * T ** 3 / 3 + a[:, 4] * T ** 4 / 4
    h_RT = (a[:, 0] * T + a[:, 1] * T ** 2 / 2 + a[:, 2] * T ** 3 / 3 + a[:, 3] * T ** 4 / 4
            + a[:, 4] * T ** 5 / 5 + a[:, 5]) / T
    s0 = rng.uniform(-2.0, 2.0, ns) + h_RT - s_var
    return case, W.MechanismTable(nu_f, nu_b, A, B, E, third, eff, np.ones(nr, dtype=bool), s0)


@pytest.mark.parametrize("dt,n_sub", [(1e-6, 8), (1e-7, 1)])
def test_higher_order_reactions_match_oracle(dt, n_sub):
    """concentration products with a species two and three times on a side
    (the molecule lists of the kernel) against the oracle's powers"""
    xf = _xf()
    case, mt = higher_order_case()
    th, g = oracle_objects(case)
    U0 = O.fill_ghosts(g, case.U)
    ref = O.fill_ghosts(g, R.react(th, _omech(mt), g, U0, dt, n_sub))
    ctx = xf.Context.from_case(case).set_reactions(mt, n_sub)
    U = ctx.state_from_numpy(U0)
    ctx.react(U, dt)
    flags = ctx.status()
    got = U.cpu().numpy()
    ctx.close()
    change = np.abs(ref[:th.ns] - U0[:th.ns]).max() / np.abs(U0[:th.ns]).max()
    err = _state_err(got, ref)
    print(f"[react] higher-order dt={dt:g} n_sub={n_sub} change {change:.2e} max err {err.max():.3e}", flush=True)
    assert flags == 0
    assert change > 1e-6
    assert err.max() <= TOL, err


def _state_err(U_gpu, U_ora):
    scale = np.abs(U_ora).reshape(U_ora.shape[0], -1).max(axis=1)
    return field_err(U_gpu, U_ora, scale)


@pytest.mark.parametrize("name", ["n9_1500K", "n9_1500K_all_reactions", "n3_dissociation"])
@pytest.mark.parametrize("dt,n_sub", [(1e-6, 16), (1e-7, 1)])
def test_reaction_step_matches_oracle(name, dt, n_sub):
    xf = _xf()
    case, mt = reacting_case(name)
    th, g = oracle_objects(case)
    U0 = O.fill_ghosts(g, case.U)
    ref = O.fill_ghosts(g, R.react(th, _omech(mt), g, U0, dt, n_sub))
    ctx = xf.Context.from_case(case).set_reactions(mt, n_sub)
    U = ctx.state_from_numpy(U0)
    ctx.react(U, dt)
    flags = ctx.status()
    got = U.cpu().numpy()
    ctx.close()
    change = np.abs(ref[:th.ns] - U0[:th.ns]).max() / np.abs(U0[:th.ns]).max()
    err = _state_err(got, ref)
    print(f"[react] {name} nr={mt.nr} dt={dt:g} n_sub={n_sub} change {change:.2e} max err {err.max():.3e}",
          flush=True)
    assert flags == 0
    assert err.max() <= TOL, err


@pytest.mark.parametrize("splitting", ["strang", "lie"])
def test_split_rk3_matches_oracle(splitting):
    xf = _xf()
    case, mt = reacting_case("n9_1500K")
    th, g = oracle_objects(case)
    Uo = O.fill_ghosts(g, case.U)
    dt = 0.4 * O.cfl_dt(th, g, Uo, 0.5)
    ctx = xf.Context.from_case(case).set_reactions(mt, 8, splitting)
    U = ctx.state_from_numpy(case.U)
    for _ in range(2):
        Uo = O.rk3_step(th, g, Uo, dt, mechanism=_omech(mt), n_sub=8, splitting=splitting)
        ctx.rk3_step(U, dt)
    assert ctx.status() == 0
    err = _state_err(U.cpu().numpy(), Uo)
    ctx.close()
    print(f"[react] rk3 {splitting} dt={dt:.3e} max err {err.max():.3e}", flush=True)
    assert err.max() <= TOL, err


def test_split_rk3_with_device_cfl_step():
    xf = _xf()
    case, mt = reacting_case("n9_1500K")
    th, g = oracle_objects(case)
    Uo = O.fill_ghosts(g, case.U)
    dt = O.cfl_dt(th, g, Uo, 0.4)
    Uo = O.rk3_step(th, g, Uo, dt, mechanism=_omech(mt), n_sub=4)
    ctx = xf.Context.from_case(case).set_reactions(mt, 4)
    U = ctx.state_from_numpy(case.U)
    dt_dev = torch.zeros(1, dtype=torch.float64, device=U.device)
    ctx.rk3_step_cfl(U, 0.4, dt_dev)
    assert abs(float(dt_dev.item()) / dt - 1.0) < 1e-13
    err = _state_err(U.cpu().numpy(), Uo)
    ctx.close()
    print(f"[react] rk3_cfl max err {err.max():.3e}", flush=True)
    assert err.max() <= TOL, err


def test_full_size_sampled_reaction_step():
    """nine-species shock-bubble at 256^3 with the synthetic mechanism and
    formation enthalpies: GPU reaction step on the whole grid, oracle on
    sampled cells"""
    xf = _xf()
    case = W.nine_species_sbi(256)
    tab = W.with_formation_enthalpies(case.thermo, 1)
    case = W.rethermo(case, tab)
    mt = W.synthetic_mechanism(W.W9, tab, 0, 12)
    th, g = oracle_objects(case)
    print("[react] full-size 256^3", flush=True)
    ctx = xf.Context.from_case(case).set_reactions(mt, 4)
    U = ctx.state_from_numpy(case.U)
    ctx.fill_ghosts(U)
    U0 = U.cpu().numpy()
    ctx.react(U, 2e-6)
    got = U.cpu().numpy()
    assert ctx.status() == 0
    ctx.close()
    del U
    rng = np.random.default_rng(7)
    nx, ny, nz = case.n
    cells = np.array([rng.integers(0, [nx, ny, nz]) for _ in range(300)] +
                     [(x, ny // 2, nz // 2) for x in range(30, 120, 3)])
    sel = (slice(None), cells[:, 2] + 3, cells[:, 1] + 3, cells[:, 0] + 3)
    Uc = U0[sel]
    ns = th.ns
    rho = Uc[:ns].sum(axis=0)
    Y = (Uc[:ns] / rho).T
    u = Uc[ns:ns + 3] / rho
    e = Uc[ns + 3] / rho - 0.5 * (u ** 2).sum(axis=0)
    Yo = R.react_cells(th, _omech(mt), rho, Y, e, 2e-6, 4)
    ref = (Yo * rho[:, None]).T
    # species absent from the whole state (most of the nine) are created in
    # traces: every partial density is judged against the largest density
    scale = np.abs(U0[:ns]).sum(axis=0).max()
    err = np.abs(got[sel][:ns] - ref).max(axis=1) / scale
    change = np.abs(ref - Uc[:ns]).max()
    print(f"[react] full-size sampled change {change:.2e} max err {err.max():.3e}", flush=True)
    assert err.max() <= TOL, err
    assert np.array_equal(got[sel][ns:], Uc[ns:])             # momentum and energy untouched


def test_reaction_refusals():
    xf = _xf()
    case, mt = reacting_case("n9_1500K")
    ctx = xf.Context.from_case(case)
    U = ctx.state_from_numpy(case.U)
    ctx.fill_ghosts(U)
    with pytest.raises(xf.XfError) as e:
        ctx.react(U, 1e-7)
    assert e.value.code == xf.XF_EUNSUPPORTED
    bad = W.MechanismTable(mt.nu_f.copy(), mt.nu_b, mt.A, mt.B, mt.E, mt.third, mt.eff, mt.reversible, mt.s0)
    bad.nu_f[0, 0] += 1                                          # no longer conserves mass
    with pytest.raises(xf.XfError) as e:
        ctx.set_reactions(bad, 4)
    assert e.value.code == xf.XF_EINVAL
    big = W.MechanismTable(mt.nu_f.copy(), mt.nu_b.copy(), mt.A, mt.B, mt.E, mt.third, mt.eff, mt.reversible, mt.s0)
    big.nu_f[0] = 0
    big.nu_b[0] = 0
    big.nu_f[0, :3] = 3                                          # nine molecules on each side, mass conserved
    big.nu_b[0, :3] = 3
    with pytest.raises(xf.XfError) as e:
        ctx.set_reactions(big, 4)
    assert e.value.code == xf.XF_EINVAL
    big.nu_f[0, 2] = 1                                           # seven on each side: accepted
    big.nu_b[0, 2] = 1
    ctx.set_reactions(big, 4)
    ctx.set_reactions(mt, 4)
    with pytest.raises(xf.XfError) as e:
        ctx.rhs_vjp(U, torch.ones_like(U))
    assert e.value.code == xf.XF_EUNSUPPORTED
    ctx.close()


def test_all_terms_together_match_oracle():
    """one split step with everything on at once: WENO7 on four ghost
    layers, GLF speeds, the positivity blend, viscous and diffusive fluxes
    and the reaction source (Strang)"""
    xf = _xf()
    case, mt = reacting_case("n9_1500K")
    case = case.with_ghosts(4)
    th, g = oracle_objects(case)
    tr = W.sampled_transport(th.ns, 0)
    otr = O.xf_viscous.Transport(tr.mu, tr.kappa, tr.D, tr.p_ref)
    Uo = O.fill_ghosts(g, case.U)
    dt = 0.3 * O.cfl_dt(th, g, Uo, 0.5)
    Uo = O.rk3_step(th, g, Uo, dt, pp=True, visc="GLF", recon="WENO7", transport=otr, mechanism=_omech(mt), n_sub=4)
    ctx = (xf.Context.from_case(case).set_reconstruction("WENO7").set_dissipation("GLF").set_positivity(True)
           .set_viscous(tr).set_reactions(mt, 4))
    U = ctx.state_from_numpy(case.U)
    ctx.rk3_step(U, dt)
    assert ctx.status() == 0
    err = _state_err(U.cpu().numpy(), Uo)
    ctx.close()
    print(f"[react] all terms (WENO7, GLF, blend, viscous, reactions) max err {err.max():.3e}", flush=True)
    assert err.max() <= TOL, err


# Mixed precision with formation enthalpies (a5 != 0) and reactions: the FP32
# face c~^2 = Gamma (H~ - |u~|^2) + sum_s Y~_s chi_s carries e_s(T~) with its
# enthalpy constant, so the cancellation is larger than on the a5 = 0 tables
# of the other mixed cases.  Declared bounds as for the other mixed cases:
# one residual within 2e-5 S_f, the state after split steps within 1e-5 of
# each field's largest magnitude (the reaction step itself runs in FP64).
@pytest.mark.parametrize("name", ["n9_1500K", "n3_dissociation"])
def test_rhs_mixed_formation_enthalpies_within_fp32_bound(name):
    from test_gpu_parity import gpu_rhs, oracle_rhs
    case, _ = reacting_case(name)
    r_gpu, flags, _ = gpu_rhs(case, "mixed")
    r_ora, aux, _ = oracle_rhs(case)
    assert flags == 0
    err = field_err(r_gpu, r_ora, aux["scale_llf"])
    print(f"[react] mixed rhs, formation enthalpies {name}: max err / S_f = {err.max():.3e}", flush=True)
    assert err.max() <= 2e-5, err


@pytest.mark.parametrize("splitting", ["strang", "lie"])
def test_split_rk3_mixed_within_fp32_bound(splitting):
    xf = _xf()
    case, mt = reacting_case("n9_1500K")
    th, g = oracle_objects(case)
    Uo = O.fill_ghosts(g, case.U)
    dt = 0.4 * O.cfl_dt(th, g, Uo, 0.5)
    ctx = xf.Context.from_case(case, "mixed").set_reactions(mt, 8, splitting)
    U = ctx.state_from_numpy(case.U)
    for _ in range(2):
        Uo = O.rk3_step(th, g, Uo, dt, mechanism=_omech(mt), n_sub=8, splitting=splitting)
        ctx.rk3_step(U, dt)
    assert ctx.status() == 0
    err = _state_err(U.cpu().numpy(), Uo)
    ctx.close()
    print(f"[react] mixed rk3 {splitting} dt={dt:.3e} max err {err.max():.3e}", flush=True)
    assert err.max() <= 1e-5, err
