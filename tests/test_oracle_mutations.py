"""The pins are strong enough: each plausible mistake planted in a copy of
the oracle source (a dropped term, a wrong sign, coefficient, index or time
level) makes at least one pin fail.  Runs on the CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests import test_oracle_pins as P

# (name, text in prs_oracle.c, replacement)
MUTATIONS = [
    ("laplacian centre coefficient", "acc -= 2.0 * p->ndim * f[i];", "acc -= 2.0 * (p->ndim + 1) * f[i];"),
    ("laplacian misses 1/dx^2", "return acc / (p->dx * p->dx);", "return acc;"),
    ("y neighbour two sites away", "if (d == 1) y = wrap(y + s, ny);", "if (d == 1) y = wrap(y + 2 * s, ny);"),
    ("damping sign", "(1.0 - delta) * pi[i]", "(1.0 + delta) * pi[i]"),
    ("damping at eta_{n+1}", "double delta = orc_delta(p, n);\n    double deta = p->deta;",
     "double delta = orc_delta(p, n + 1);\n    double deta = p->deta;"),
    ("damping without m", "return 0.5 * p->alpha * (p->deta / orc_eta(p, n)) * p->m;",
     "return 0.5 * p->alpha * (p->deta / orc_eta(p, n));"),
    ("force sign", "return 4.0 * p->V0 * f * q / (p->phi0 * p->phi0);",
     "return -4.0 * p->V0 * f * q / (p->phi0 * p->phi0);"),
    ("force coefficient", "return 4.0 * p->V0 * f * q / (p->phi0 * p->phi0);",
     "return 2.0 * p->V0 * f * q / (p->phi0 * p->phi0);"),
    ("drift with the undamped kick", "phi_next[i] = phi[i] + deta * pi[i];          /* Eq. (5) */",
     "phi_next[i] = phi[i] + deta * kick;"),
    ("sign test phi > 0", "int si = phi[i] >= 0.0;", "int si = phi[i] > 0.0;"),
    ("area weight without sqrt", "double w = gabs > 0.0 ? sqrt(gsq) / gabs : 1.0;",
     "double w = gabs > 0.0 ? gsq / gabs : 1.0;"),
    ("area element dx^D", "double dA = pow(p->dx, p->ndim - 1);", "double dA = pow(p->dx, p->ndim);"),
    ("kinetic energy without 1/2", "if (V > 0.0) ek += 0.5 * pi[i] * pi[i] / V;",
     "if (V > 0.0) ek += pi[i] * pi[i] / V;"),
    ("wall sites from forward links only", "if (sb != si) wall = 1;", ""),
    ("adjoint V'' sign", "mu[i] = mu[i] + b * (lw - A * d2V(p, ph[i]) * w[i]);",
     "mu[i] = mu[i] + b * (lw + A * d2V(p, ph[i]) * w[i]);"),
    ("adjoint drops the damping factor", "for (int64_t i = 0; i < N; ++i) nu[i] = a * w[i];",
     "for (int64_t i = 0; i < N; ++i) nu[i] = w[i];"),
    ("adjoint V0 derivative sign", "G -= b * g;", "G += b * g;"),
    ("force without the scale-factor power", "deta * (lap - A * dV(p, phi[i]))", "deta * (lap - dV(p, phi[i]))"),
    ("force with a^(beta/2)", "return pow(pow(orc_eta(p, n) / p->eta0, p->m), p->beta);",
     "return pow(pow(orc_eta(p, n) / p->eta0, p->m), 0.5 * p->beta);"),
    ("wall potential energy without a^beta", "double V = A * Vpot(p, phi[i]);", "double V = Vpot(p, phi[i]);"),
    ("area gradient by forward difference", "double g = (phi[jf] - phi[jb]) / (2.0 * p->dx);",
     "double g = (phi[jf] - phi[i]) / p->dx;"),
    ("area weight at the upper endpoint",
     "            if (crossings) {\n                double w = gabs > 0.0 ? sqrt(gsq) / gabs : 1.0;\n"
     "                area += (double)crossings * w;\n            }",
     "            for (int d2 = 0; d2 < p->ndim; ++d2) {\n"
     "                int64_t j = neighbour(p, x, y, z, d2, +1);\n"
     "                if (si == (phi[j] >= 0.0)) continue;\n"
     "                int64_t jx = j % nx, jy = (j / nx) % ny, jz = j / (nx * ny);\n"
     "                double s2 = 0.0, s1 = 0.0;\n"
     "                for (int e = 0; e < p->ndim; ++e) {\n"
     "                    double h = phi[neighbour(p, jx, jy, jz, e, +1)] - phi[neighbour(p, jx, jy, jz, e, -1)];\n"
     "                    s2 += h * h; s1 += fabs(h);\n"
     "                }\n"
     "                area += s1 > 0.0 ? sqrt(s2) / s1 : 1.0;\n"
     "            }"),
    ("adjoint V'' without a^beta", "mu[i] = mu[i] + b * (lw - A * d2V(p, ph[i]) * w[i]);",
     "mu[i] = mu[i] + b * (lw - d2V(p, ph[i]) * w[i]);"),
]


def pins():
    """Fast subset of the pins, as (name, callable)."""
    return [
        ("P1 vacuum", lambda: P.test_p1_vacuum_is_static_bitwise((8, 6), 1.0)),
        ("P3 translation", lambda: P.test_p3_translation_bitwise((20, 14), (7, 3))),
        ("P5 kink 2D", lambda: P.test_p5_static_kink_pair((128, 4))),
        ("P6 energy", P.test_p6_kink_energy_bounded),
        ("P7 free 2D", lambda: P.test_p7_free_dispersion((24, 16), (3, 2), 0.5, 0.1)),
        ("P7 vacuum", lambda: P.test_p7_vacuum_dispersion((16, 12), (2, 1))),
        ("P8 damping", lambda: P.test_p8_damping_power_law(3.0, 2.0)),
        ("P9 links", lambda: P.test_p9_link_counts_brute_force((4, 3), None)),
        ("P9 zero", P.test_p9_zero_tiebreak),
        ("P10 diagonal", lambda: P.test_p10_diagonal_walls((32, 32))),
        ("P10 dx", P.test_p10_area_scales_with_dx),
        ("P10 oblique", lambda: P.test_p10_oblique_sine_walls(32)),
        ("P10 lower endpoint", lambda: P.test_p10_weight_at_lower_endpoint((16, 12))),
        ("P11 velocity", lambda: P.test_p11_boosted_wall_velocity((64, 8), 0.3)),
        ("P11 wall sites", P.test_p11_mean_over_wall_sites_only),
        ("P13 adjoint", lambda: P.test_adjoint_matches_finite_differences(16, 3.0, 0.0)),
        ("P13 adjoint beta", lambda: P.test_adjoint_matches_finite_differences(24, 2.0, 2.0)),
        ("P14 homogeneous", P.test_p14_beta_force_homogeneous_mode),
        ("P14 velocity", lambda: P.test_p14_boosted_wall_velocity_with_beta((64, 8), 0.3)),
    ]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_reject_mutation(tmp_path, name, old, new):
    src = O.source_text()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    lib = O.build_variant(src.replace(old, new), str(tmp_path / "mutant.so"))
    caught = []
    with O.using_library(lib):
        for pin, fn in pins():
            try:
                fn()
            except AssertionError:
                caught.append(pin)
    assert caught, "no pin detects: " + name
