"""Planted mistakes: each mutant of the oracle source must fail at least one pin.

Every case copies ``oracle/sphx_oracle.c``, applies one plausible mistake (a
dropped term, a wrong sign, a wrong mean, a transposed exponent, a missing self
term, a wrong constant, a broken minimal image, a wrong integrator stage),
compiles it into a temporary library on the CPU and runs the pins that should
catch it against that library.  The product code is never touched.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sphx_oracle.c")

MUTANTS = {
    "pressure_drops_Pj": ("const double cp = (c->m[i] * c->m[j]) * (Ai + Aj);",
                          "const double cp = (c->m[i] * c->m[j]) * (Ai + Ai);",
                          "antisymmetric or momentum"),
    "viscosity_sign": ("cv = Vj * (2.0 * nuij) * lap;", "cv = -Vj * (2.0 * nuij) * lap;",
                       "viscosity_linear_shear"),
    "arithmetic_mean": ("double nuij = (pi->nu + pj->nu) > 0.0 ? 2.0 * pi->nu * pj->nu / (pi->nu + pj->nu) : 0.0;",
                        "double nuij = 0.5 * (pi->nu + pj->nu);", "harmonic_mean"),
    "colour_sigma_i_inverted": ("for (int d = 0; d < 3; ++d) gi[d] = si * s[d];",
                                "for (int d = 0; d < 3; ++d) gi[d] = s[d] / si;",
                                "colour_gradient"),
    "renorm_without_self": ("double num = c->m[i] * w0;                 /* j = i */",
                            "double num = 0.0 * w0;", "renormalisation"),
    "kernel_gradient_constant": ("return -5.0 * kernel_alpha(dim, h) / (h * h) * t * t * t;",
                                 "return -4.0 * kernel_alpha(dim, h) / (h * h) * t * t * t;",
                                 "kernel_gradient"),
    "continuity_mass_weights": ("o->cont = (c->p.cont_form == 1 ? c->m[j] : Vj) * udg;",
                                "o->cont = c->m[j] * udg;", "continuity or volume_form"),
    "tension_sign": ("        o->ms[a] = s;", "        o->ms[a] = -s;", "circle_static"),
    "tensor_fixed_d3": ("double iso = (a == b && a < dim) ? gn * gn / (double)dim : 0.0;",
                        "double iso = (a == b && a < dim) ? gn * gn / 3.0 : 0.0;", "traceless"),
    "min_image_broken": ("if (v > 0.5 * L) v -= L;", "if (v > 2.0 * L) v -= L;",
                         "neighbour or lattice"),
    "corrector_uses_un": ("xi[d] = xn[3 * i + d] + fdt * c->u[3 * i + d];",
                          "xi[d] = xn[3 * i + d] + fdt * un[3 * i + d];", "free_fall"),
    "eos_beta_missing_gamma": ("double beta = rho0 * c0 * c0 / gamma;          /* Eq. (4) */",
                               "double beta = rho0 * c0 * c0;", "tait"),
    "renorm_rho_i_for_rho_j": ("den += c->m[j] / c->rho[j] * w;", "den += c->m[j] / c->rho[i] * w;",
                               "renormalisation"),
    "renorm_mass_of_i": ("num += c->m[j] * w;", "num += c->m[i] * w;", "renormalisation"),
    "renorm_wrong_weight": ("double w = so_kernel_w(dim, h, sqrt(pair_vector(c, i, j, r)));",
                            "double w = so_kernel_w(dim, h, 0.9 * sqrt(pair_vector(c, i, j, r)));",
                            "renormalisation"),
    "piston_drops_cos_phi": ("(cos(p->piston_w[k] * te + p->piston_phi[k]) - cos(p->piston_phi[k]))",
                             "(cos(p->piston_w[k] * te + p->piston_phi[k]) - 1.0)", "piston or wavemaker"),
    "piston_phase_sign": ("(cos(p->piston_w[k] * te + p->piston_phi[k]) - cos(p->piston_phi[k]))",
                          "(cos(p->piston_w[k] * te - p->piston_phi[k]) - cos(p->piston_phi[k]))",
                          "piston or wavemaker"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught_by_a_pin(name, tmp_path):
    old, new, selector = MUTANTS[name]
    with open(SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I", os.path.join(ROOT, "oracle"), "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, SPHX_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", selector],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout + r.stderr
    assert r.returncode != 0, f"mutant {name} survived the pins selected by '{selector}'"
