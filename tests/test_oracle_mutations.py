"""Planted mistakes: each test builds a copy of an oracle module with one
plausible error (a flipped sign, a dropped factor, a swapped operand) and
checks that at least one pin fails on it.  This shows the pins constrain the
oracle's arithmetic, not just its plumbing.  Everything runs on the CPU.
"""
import importlib
import os
import sys
import types

import pytest

import oracle
import tests.test_oracle_fft as pins_fft
import tests.test_oracle_physics as pins_phys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def mutated(modname, old, new):
    path = os.path.join(ROOT, "oracle", modname + ".py")
    with open(path) as f:
        src = f.read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    src = src.replace(old, new, 1)
    mod = types.ModuleType(f"oracle.{modname}")
    mod.__package__ = "oracle"
    mod.__file__ = path
    exec(compile(src, path, "exec"), mod.__dict__)
    return mod


def must_fail(pin, *args):
    with pytest.raises(AssertionError):
        pin(*args)


QG_MUTATIONS = [
    ("beta sign", "- p.beta * 1j * g.kx * psih", "+ p.beta * 1j * g.kx * psih",
     lambda: pins_phys.test_single_shell_rk4_exact("none", 0.0)),
    ("jacobian sign", "J = u * wx + v * wy", "J = u * wx - v * wy",
     pins_phys.test_jacobian_two_modes_closed_form),
    ("strain factor", "4.0 * pxy ** 2 + pd ** 2", "2.0 * pxy ** 2 + pd ** 2",
     pins_phys.test_poisson_and_second_derivatives_closed_form),
    ("test ratio power", "power = 2 if kind == \"dsmag\" else 3",
     "power = 3 if kind == \"dsmag\" else 2",
     lambda: pins_phys.test_dynamic_coefficient_inside_test_filter("dsmag", 2)),
    ("penalization operands", "m.Ex * v - m.Ey * u", "m.Ex * u - m.Ey * v",
     pins_phys.test_island_interior_decay_and_inflow_vorticity),
    ("rk4 weight", "k1 + 2.0 * k2 + 2.0 * k3 + k4", "k1 + k2 + 2.0 * k3 + k4",
     lambda: pins_phys.test_single_shell_rk4_exact("none", 0.0)),
    ("divergence index", "1j * g.kx * hxh + 1j * g.ky * hyh", "1j * g.kx * hxh + 1j * g.kx * hyh",
     lambda: pins_phys.test_eddy_viscosity_dissipates_enstrophy_exactly("smag")),
    ("dropped test filter", "- g.T * Jh", "- Jh",
     lambda: pins_phys.test_dynamic_coefficient_inside_test_filter("dleith", 3)),
    ("viscosity sign", "- (g.k2 * m.inv_re + p.mu) * wh", "+ (g.k2 * m.inv_re + p.mu) * wh",
     lambda: pins_phys.test_single_shell_rk4_exact("none", 0.0)),
    ("pointwise clip of the product", "np.mean(np.maximum(H, 0.0) * M)", "np.mean(np.maximum(H * M, 0.0))",
     lambda: pins_phys.test_pointwise_clip_reading("dleith")),
    ("diagnostics nu_e mean of the magnitude", "float(nu.mean())", "float(np.abs(nu - nu.mean()).mean())",
     lambda: pins_phys.test_diag_eddy_viscosity_field_and_statistics("leith")),
    ("diagnostics nu_e statistics swapped", "float(nu.min()), float(nu.mean()), float(nu.max())",
     "float(nu.min()), float(nu.max()), float(nu.mean())",
     lambda: pins_phys.test_diag_eddy_viscosity_field_and_statistics("dsmag")),
    ("diagnostics CFL without the time step", "* p.dt / g.delta", "/ g.delta",
     pins_phys.test_oversized_dt_drives_cfl_past_one_until_nonfinite),
]


@pytest.mark.parametrize("name,old,new,pin", QG_MUTATIONS, ids=[m[0] for m in QG_MUTATIONS])
def test_qg_mutation_is_caught(monkeypatch, name, old, new, pin):
    mod = mutated("qg", old, new)
    monkeypatch.setattr(pins_phys, "qg", mod)
    must_fail(pin)


def test_fft_twiddle_sign_is_caught(monkeypatch):
    mod = mutated("fft", "ang = sign * 2.0 * np.pi * k / (2 * L)",
                  "ang = -sign * 2.0 * np.pi * k / (2 * L)")
    monkeypatch.setattr(pins_fft, "F", mod)
    must_fail(pins_fft.test_1d_against_definition, 8)


def test_fft_hermitian_weight_is_caught(monkeypatch):
    mod = mutated("fft", "full[..., 0] = cols[..., 0].real", "full[..., 0] = 2 * cols[..., 0].real")
    monkeypatch.setattr(pins_fft, "F", mod)
    must_fail(pins_fft.test_irfft2_against_definition, 8, 8)


import tests.test_oracle_ab2cn as pins_ab2  # noqa: E402

AB2CN_MUTATIONS = [
    ("ab2 weights", "dt * (1.5 * N - 0.5 * Nm)", "dt * (1.0 * N - 0.0 * Nm)",
     pins_ab2.test_ab2_advection_by_the_inflow),
    ("crank-nicolson half", "wh * (1.0 + 0.5 * dt * L)", "wh * (1.0 + dt * L)",
     lambda: pins_ab2.test_crank_nicolson_single_mode(50.0, 0.3, 2.0)),
    ("penalty curl sign", "- 1j * g.ky * g.spec(m.chi * u)", "+ 1j * g.ky * g.spec(m.chi * u)",
     pins_ab2.test_ab2_brinkman_constant_mask),
    ("velocity history", "1.5 * u - 0.5 * um", "1.5 * u - 0.5 * u",
     pins_ab2.test_ab2_brinkman_constant_mask),
    ("sponge history", "(1.5 * ws - 0.5 * wss)", "(1.5 * ws - 0.5 * ws)",
     pins_ab2.test_ab2_sponge_constant_profile),
    ("rossby sign", "+ 1j * p.beta * g.kx * g.inv_k2", "- 1j * p.beta * g.kx * g.inv_k2",
     pins_ab2.test_rossby_phase_and_modulus),
]


@pytest.mark.parametrize("name,old,new,pin", AB2CN_MUTATIONS, ids=[m[0] for m in AB2CN_MUTATIONS])
def test_ab2cn_mutation_is_caught(monkeypatch, name, old, new, pin):
    mod = mutated("ab2cn", old, new)
    monkeypatch.setattr(pins_ab2, "ab2cn", mod)
    must_fail(pin)


import tests.test_oracle_les as pins_les  # noqa: E402

LES_MUTATIONS = [
    ("gaussian width not squared", "k2 * (delta * dfr) ** 2 / 6.0", "k2 * (delta * dfr) / 6.0",
     lambda: pins_les.test_gaussian_equals_physical_convolution(2)),
    ("coarse rescaling", "ch / (delta * delta)", "ch / delta",
     pins_les.test_cutoff_edges_and_single_mode_amplitude),
    ("cut-off radius", "kc = np.pi / (delta * dfr)", "kc = 1.1 * np.pi / (delta * dfr)",
     pins_les.test_cutoff_edges_and_single_mode_amplitude),
    ("pcc centring", "dy = y - y.mean()", "dy = y",
     pins_les.test_pcc_against_numpy_and_affine),
    ("penalty forcing sign", "G = G + (1.0 / p.eta)", "G = G - (1.0 / p.eta)",
     pins_les.test_ideal_sgs_penalty_and_sponge_commutators_closed_form),
    ("curl operands", "g.spec(m.chi * v) - 1j * g.ky * g.spec(m.chi * u)",
     "g.spec(m.chi * u) - 1j * g.ky * g.spec(m.chi * v)",
     pins_les.test_ideal_sgs_penalty_and_sponge_commutators_closed_form),
    ("dropped sponge rate", "G = G + p.sponge_sigma * g.D", "G = G + g.D",
     pins_les.test_ideal_sgs_penalty_and_sponge_commutators_closed_form),
    ("commutator order", "(advective_forcing(wbar_d, m_les) - Gbar)", "(Gbar - advective_forcing(wbar_d, m_les))",
     pins_les.test_ideal_sgs_two_modes_closed_form),
    ("no projection on D", "Pi = gl.D * (advective_forcing", "Pi = (advective_forcing",
     pins_les.test_ideal_sgs_is_projected_on_the_les_two_thirds_set),
    ("model without coefficient", 'g.phys(out["C"] * out["Qh"])', 'g.phys(out["Qh"])',
     lambda: pins_les.test_model_sgs_enstrophy_identity("leith", 3)),
]


@pytest.mark.parametrize("name,old,new,pin", LES_MUTATIONS, ids=[m[0] for m in LES_MUTATIONS])
def test_les_mutation_is_caught(monkeypatch, name, old, new, pin):
    mod = mutated("les", old, new)
    monkeypatch.setattr(pins_les, "les", mod)
    must_fail(pin)


import tests.test_oracle_adjoint as pins_adj  # noqa: E402

ADJ_MUTATIONS = [
    ("test level without T", "g.T * transport_adjoint(g.T * x, a, r * b, kind, m)",
     "g.T * transport_adjoint(x, a, r * b, kind, m)",
     lambda: pins_adj.test_dynamic_rhs_adjoint_central_fd("dleith")),
    ("M factor in grad C", "(fw[\"Hh\"] - 2.0 * C * fw[\"Mh\"])", "(fw[\"Hh\"] - C * fw[\"Mh\"])",
     lambda: pins_adj.test_dynamic_rhs_adjoint_central_fd("dsmag")),
    ("test ratio power in grad C", "** (2 if p.closure == \"dsmag\" else 3)", "** (3 if p.closure == \"dsmag\" else 2)",
     lambda: pins_adj.test_dynamic_rhs_adjoint_central_fd("dleith")),
    ("flux cotangent sign", "gx = g.phys(-1j * g.kx * g.D * cQ)", "gx = g.phys(1j * g.kx * g.D * cQ)",
     lambda: pins_adj.test_dynamic_rhs_adjoint_central_fd("dsmag")),
]


@pytest.mark.parametrize("name,old,new,pin", ADJ_MUTATIONS, ids=[m[0] for m in ADJ_MUTATIONS])
def test_adjoint_mutation_is_caught(monkeypatch, name, old, new, pin):
    mod = mutated("adjoint", old, new)
    monkeypatch.setattr(pins_adj, "adj", mod)
    must_fail(pin)
