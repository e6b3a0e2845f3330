"""Planted mistakes in the oracle source must break at least one pin.

Each case copies oracle/fe_oracle.c, applies one plausible slip (a dropped
term, a wrong sign or index, a transposed operand, the wrong boundary), builds
the copy into a temporary library and routes the oracle wrapper to it.  The
named pin must then report a discrepancy far above its tolerance, which shows
the pins are sharp enough to catch that class of mistake.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from test_oracle_pins import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "fe_oracle.c")

# (name, original text, mutated text, pin call, threshold it must exceed)
MUTANTS = [
    ("anscombe_offset", "sqrt(y[p] + 3.0 / 8.0)", "sqrt(y[p] + 1.0 / 8.0)",
     pins.anscombe_zero, 1e-3),
    ("inverse_coefficient", "(11.0 / 8.0) / (z * z)", "(11.0 / 4.0) / (z * z)",
     pins.inverse_derivative, 1e-3),
    ("inverse_coefficient_unbiased", "(11.0 / 8.0) / (z * z)", "(11.0 / 4.0) / (z * z)",
     pins.inverse_unbiased, 0.05),
    ("inverse_sign", "+ 0.25 * c / z", "- 0.25 * c / z",
     pins.inverse_derivative, 1e-3),
    ("zero_padding",
     "e[i * We + j] = u[sym_index(i - r, H) * W + sym_index(j - r, W)];",
     "e[i * We + j] = (i < r || i >= H + r || j < r || j >= W + r) ? 0.0 : u[(i - r) * W + (j - r)];",
     pins.constant_kernel, 1e-3),
    ("zero_padding_scipy",
     "e[i * We + j] = u[sym_index(i - r, H) * W + sym_index(j - r, W)];",
     "e[i * We + j] = (i < r || i >= H + r || j < r || j >= W + r) ? 0.0 : u[(i - r) * W + (j - r)];",
     pins.forward_vs_scipy, 1e-3),
    ("convolution_not_correlation",
     "const double *er = e + (y + a) * We + b;\n                    for (long x = 0; x < W; ++x) row[x] += kab * er[x];",
     "const double *er = e + (y + m - 1 - a) * We + (m - 1 - b);\n                    for (long x = 0; x < W; ++x) row[x] += kab * er[x];",
     pins.adjoint_identity, 1e-3),
    ("transposed_taps",
     "const double kab = ki[a * m + b];\n                    const double *er",
     "const double kab = ki[b * m + a];\n                    const double *er",
     pins.forward_vs_scipy, 1e-3),
    ("adjoint_unfolded_columns",
     "g[y * W + sym_index(t - r, W)] += G[s * We + t];",
     "if (t >= r && t < W + r) g[y * W + t - r] += G[s * We + t];",
     pins.adjoint_identity, 1e-3),
    ("adjoint_unfolded_rows",
     "const long cand[3] = { r - 1 - y, y + r, 2 * (long)H - 1 - y + r };",
     "const long cand[3] = { -1, y + r, -1 };",
     pins.adjoint_vs_dense, 1e-3),
    ("adjoint_wrong_direction",
     "const double *wr = wz + (s - a + P) * Wz + (P - b);",
     "const double *wr = wz + (s + a - P) * Wz + (b - P) + 2 * P;",
     pins.adjoint_identity, 1e-3),
    ("influence_factor", "return 2.0 * z / (1.0 + z * z);", "return z / (1.0 + z * z);",
     pins.rho_prime_fd, 1e-3),
    ("influence_factor_grad", "return 2.0 * z / (1.0 + z * z);", "return z / (1.0 + z * z);",
     pins.grad_prior_fd, 1e-3),
    ("potential_dropped_weight", "e += alpha[i] * ordered_sum(zi, H, W);", "e += ordered_sum(zi, H, W);",
     pins.grad_prior_fd, 1e-3),
    ("idiv_prox_term", "sqrt(a * a + 4.0 * tl * v)", "sqrt(a * a + 2.0 * tl * v)",
     pins.prox_optimality, 1e-3),
    ("quadratic_prox_denominator", "return (ut + tl * v) / (1.0 + tl);",
     "return (ut + tl * v) / (1.0 + 2.0 * tl);", pins.prox_optimality, 1e-3),
    ("inertia_sign", "+ gamma * (u[p] - u_prev[p])", "- gamma * (u[p] - u_prev[p])",
     lambda: pins.ipiano_vs_dense(2, iters=20), 1e-6),
    ("step_scale", "u[p] - tau * g[p]", "u[p] - 0.5 * tau * g[p]",
     lambda: pins.ipiano_vs_dense(1, iters=20), 1e-6),
    ("data_gradient_dropped", "for (long p = 0; p < n; ++p) grad[p] += gd[p];",
     "for (long p = 0; p < n; ++p) grad[p] += 0.0 * gd[p];", pins.grad_full_fd, 1e-3),
    ("idiv_energy_log", "t[p] = u[p] - v[p] * log(u[p]);", "t[p] = u[p] - log(u[p]);",
     pins.grad_full_fd, 1e-3),
    ("idiv_energy_linear_term", "t[p] = u[p] - v[p] * log(u[p]);",
     "t[p] = 0.5 * u[p] - v[p] * log(u[p]);", pins.idiv_energy_vs_kl, 1e-6),
    ("energy_log_argument", "log(1.0 + z * z)", "log(2.0 + z * z)",
     pins.energy_prior_vs_dense, 1e-3),
    ("quadratic_energy_half", "0.5 * d * d", "d * d",
     pins.energy_quadratic_offset, 1e-3),
    ("power_iteration_weights",
     "for (long p = 0; p < n; ++p) z[(size_t)i * n + p] *= alpha[i];",
     "for (long p = 0; p < n; ++p) z[(size_t)i * n + p] *= 1.0;",
     pins.power_iteration_vs_eig, 1e-3),
    ("bin3_zero_padding",
     "s += y[sym_index(3 * i + a, H) * W + sym_index(3 * j + b, W)];",
     "s += (3 * i + a < H && 3 * j + b < W) ? y[(3 * i + a) * W + 3 * j + b] : 0.0;",
     pins.bin3_vs_padded, 0.5),
    ("bin3_short_block", "for (int a = 0; a < 3; ++a)\n                for (int b = 0; b < 3; ++b)",
     "for (int a = 0; a < 2; ++a)\n                for (int b = 0; b < 3; ++b)",
     pins.bin3_vs_padded, 0.5),
    ("upsample3_centre_offset", "double fy = (y - 1) / 3.0;", "double fy = y / 3.0;",
     pins.upsample3_centres, 1e-6),
    ("upsample3_no_division", "x[y * W + xx] = v / 9.0;", "x[y * W + xx] = v;",
     pins.upsample3_centres, 1e-6),
    ("upsample3_swapped_weights",
     "((1.0 - wx) * xb[i0 * Wb + j0] + wx * xb[i0 * Wb + j1])",
     "(wx * xb[i0 * Wb + j0] + (1.0 - wx) * xb[i0 * Wb + j1])",
     pins.upsample3_vs_scipy, 1e-6),
]


@pytest.fixture(scope="module")
def builder(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    src = open(SRC).read()

    def build(name, old, new):
        assert src.count(old) >= 1, "mutation anchor not found: " + name
        path = d / (name + ".c")
        path.write_text(src.replace(old, new, 1))
        lib = d / ("lib" + name + ".so")
        subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", str(lib), str(path),
                               "-lm"])
        return str(lib)
    yield build
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("case", MUTANTS, ids=[c[0] for c in MUTANTS])
def test_planted_mistake_is_caught(builder, case):
    name, old, new, pin, threshold = case
    lib = builder(name, old, new)
    with oracle.use_library(lib):
        with np.errstate(all="ignore"):
            try:
                value = pin()
            except Exception:  # a mutant that crashes a solve is also caught
                value = np.inf
    assert not (value <= threshold), (name, value)
