"""The oracle's pins have teeth: each plausible mistake planted in a copy of
the oracle source (on the CPU) makes the pin suite fail.

Each mutation is (original text, replacement, which occurrence).  The
mutated copy is compiled into a temporary library and the pins are run
against it in a subprocess through DNNMG_ORACLE_LIB; the mutants run in
parallel, once per module.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dnnmg_oracle.c")

MUTATIONS = {
    "mass_sign": ("(uq[c] - vq[c])", "(vq[c] - uq[c])", 0),
    "drop_convection": ("- N[a] * conv[c]", "- 0.0 * conv[c]", 0),
    "convection_transposed": ("vq[0] * gv[c][0] + vq[1] * gv[c][1]", "vq[0] * gv[0][c] + vq[1] * gv[1][c]", 0),
    "diffusion_sign": ("- nu * (dNx[a]", "+ nu * (dNx[a]", 0),
    "pressure_sign": ("+ pq * dphi_c", "- pq * dphi_c", 0),
    "pressure_component": ("(c == 0) ? dNx[a] : dNy[a]", "(c == 0) ? dNy[a] : dNx[a]", 0),
    "inverse_jacobian": ("(yt * dNs[k] - ys * dNt[k])", "(yt * dNs[k] - xt * dNt[k])", 0),
    "gauss_points": ("0.5 / sqrt(3.0)", "0.5 / sqrt(2.0)", 0),
    "gru_update_swapped": ("z[k] * he[k] + (1.0 - z[k]) * tanh(ah)", "(1.0 - z[k]) * he[k] + z[k] * tanh(ah)", 0),
    "gru_no_reset": ("ah += Uh[(size_t)k * H + m] * rh[m]", "ah += Uh[(size_t)k * H + m] * he[m]", 0),
    "gru_U_transposed": ("az += Uz[(size_t)k * H + m] * he[m]", "az += Uz[(size_t)m * H + k] * he[m]", 0),
    "mlp_no_relu": ("a[k] = s > 0.0 ? s : 0.0;", "a[k] = s;", 0),
    "prolong_axes_swapped": ("q1_shape((double)a / n, (double)b / n, N);", "q1_shape((double)b / n, (double)a / n, N);", 1),
    "restrict_corner_order": ("coarse[ncomp * c[k] + d] += N[k]", "coarse[ncomp * c[3 - k] + d] += N[k]", 0),
    "average_fixed_divisor": ("s[0] / cnt", "s[0] / 4", 0),
    "input_component": ("x[2 * nf + 2 * l] = D[2 * f];", "x[2 * nf + 2 * l] = D[2 * f + 1];", 0),
    "aspect_inverted": ("f[2] = hx / hy;", "f[2] = hy / hx;", 0),
    "features_hx_hy_swapped": ("f[0] = hx; f[1] = hy;", "f[0] = hy; f[1] = hx;", 0),
    "features_hx_one_edge": ("hx = 0.5 * (hypot(c10[0] - c00[0], c10[1] - c00[1]) +",
                             "hx = 0.5 * (hypot(c11[0] - c01[0], c11[1] - c01[1]) +", 0),
    "lumped_mass": ("Mu[2 * node[a] + c] += wd * N[a] * uq[c];", "Mu[2 * node[a] + c] += wd * 0.25 * uq[c];", 0),
    "mask_wrong_axis": ("((dir & 4u) && J == 0)", "((dir & 4u) && I == 0)", 0),
    "state_without_correction": ("uprev[f] = Pv[f] + Dbar[f];", "uprev[f] = Pv[f];", 0),
    # theta scheme (Crank-Nicolson)
    "theta_defect_sign": ("(1.0 - theta) * (Tv[2 * f + c] - Tu[2 * f + c])",
                          "(1.0 - theta) * (Tu[2 * f + c] - Tv[2 * f + c])", 0),
    "theta_defect_weight": ("(1.0 - theta) * (Tv[2 * f + c]", "theta * (Tv[2 * f + c]", 0),
    "theta_rhs_sign": ("bL[c] -= (1.0 - theta) * RT[c];", "bL[c] += (1.0 - theta) * RT[c];", 0),
    "transport_no_viscosity": ("double r = N[a] * conv + nu * (dNx[a]", "double r = N[a] * conv + 0.0 * (dNx[a]", 0),
    "transport_convection_transposed": ("double conv = wq[0] * gw[c][0] + wq[1] * gw[c][1];",
                                        "double conv = wq[0] * gw[0][c] + wq[1] * gw[1][c];", 0),
    # the paper's network form
    "continuity_sign": ("Rp[node[a]] -= wd * div * N[a];", "Rp[node[a]] += wd * div * N[a];", 0),
    "continuity_dy_for_vx": ("div += v[2 * node[k]] * (yt * dNs[k] - ys * dNt[k]) / det +",
                             "div += v[2 * node[k]] * (-xt * dNs[k] + xs * dNt[k]) / det +", 0),
    "paper_aspect_pairing": ("o[4] = h0 / h1; o[5] = h2 / h3;", "o[4] = h0 / h3; o[5] = h2 / h1;", 0),
    "paper_angle_corner": ("o[9] = corner_angle(c10, c11, c00);", "o[9] = corner_angle(c11, c10, c01);", 0),
    "peclet_area_not_size": ("double q = sqrt(0.5 * fabs(d1x * d2y - d1y * d2x));",
                             "double q = 0.5 * fabs(d1x * d2y - d1y * d2x);", 0),
    "paper_input_rp_node": ("x[2 * nf + l] = Rp[f];", "x[2 * nf + l] = Rp[f > 0 ? f - 1 : f];", 0),
    "gru_reset_after_before": ("tanh(wx + r[k] * uh)", "tanh(wx + uh)", 0),
    "conv_adjoint_direction": ("int rr = r - dr, cc = c - dc;", "int rr = r + dr, cc = c + dc;", 0),
    "vertex_block_transposed": ("conv_block(2, nf, WV, img, a);", "conv_block(nf, 2, WV, img, a);", 0),
    "conv_head_no_output_weights": ("for (int o = 0; o < nout; ++o) de[o] *= wf[o];", "(void)wf;", 0),
    # unstructured meshes
    "umesh_edge_from_own_end": ("int t = p < q ? along : n - along;", "int t = along;", 0),
    "umesh_no_transfinite_blend": ("fxy[2 * f + c] = (1 - eta) * Bp[c] + eta * Tp[c] + (1 - xi) * Lp[c] + xi * Rp[c] - bil;",
                                   "fxy[2 * f + c] = bil;", 0),
    "umesh_arc_as_chord": ("out[0] = cx + r * cos(ta + s * d);\n    out[1] = cy + r * sin(ta + s * d);",
                           "out[0] = (1.0 - s) * A[0] + s * B[0];\n    out[1] = (1.0 - s) * A[1] + s * B[1];", 0),
    "u_average_fixed_divisor": ("Dbar[2 * f] /= cnt[f];", "Dbar[2 * f] /= 4;", 0),
    "u_restrict_corner_order": ("coarse[ncomp * elems[4 * e + k] + c] += N[k] * fine[ncomp * f + c];",
                                "coarse[ncomp * elems[4 * e + k] + c] += N[3 - k] * fine[ncomp * f + c];", 0),
    "u_features_hx_edges": ("double hx = 0.5 * (hypot(c1[0] - c0[0], c1[1] - c0[1]) + hypot(c2[0] - c3[0], c2[1] - c3[1]));",
                            "double hx = 0.5 * (hypot(c1[0] - c0[0], c1[1] - c0[1]) + hypot(c2[0] - c1[0], c2[1] - c1[1]));", 0),
    "u_mask_without_ends": ("            for (int t = 0; t <= n; ++t) {\n                int a = k == 0 || k == 2",
                            "            for (int t = 1; t < n; ++t) {\n                int a = k == 0 || k == 2", 0),
    # FP8 E4M3 operand form
    "e4m3_ties_away": ("rint((ldexp(a, -e) - 1.0) * 8.0)", "round((ldexp(a, -e) - 1.0) * 8.0)", 0),
    "e4m3_truncate": ("rint((ldexp(a, -e) - 1.0) * 8.0)", "floor((ldexp(a, -e) - 1.0) * 8.0)", 0),
    "e4m3_bias8": ("((unsigned)(e + 7) << 3)", "((unsigned)(e + 8) << 3)", 0),
    "e4m3_subnormal_exponent": ("ldexp((double)m / 8.0, -6)", "ldexp((double)m / 8.0, -7)", 0),
    "fp8_scale_240": ("const float r = 448.0f / m;", "const float r = 240.0f / m;", 0),
    "gru_fp8_state_unscaled": ("(double)sh * qdot(H, qh, b + nin)", "qdot(H, qh, b + nin)", 0),
    "gru_fp8_scales_swapped": ("(double)sx * qdot(nin, qx, b) + (double)sh", "(double)sh * qdot(nin, qx, b) + (double)sx", 0),
    "gru_fp8_reset_on_state": ("(double)sUh[k] * (double)srh * qdot(H, qrh, qUh", "(double)sUh[k] * (double)sh * qdot(H, qh, qUh", 0),
    "mlp_fp8_no_relu": ("a[k] = t > 0.0 ? t : 0.0;", "a[k] = t;", 0),
}


def _mutate(text, old, new, occ):
    idx = -1
    for _ in range(occ + 1):
        idx = text.index(old, idx + 1)
    return text[:idx] + new + text[idx + len(old):]


def _run_mutant(name, workdir):
    """Compile the mutant and run the pin suites against it; returns the
    pytest exit status and the tail of its output, or the exception."""
    try:
        old, new, occ = MUTATIONS[name]
        os.makedirs(workdir, exist_ok=True)
        msrc = os.path.join(workdir, "mutant.c")
        with open(msrc, "w") as fh:
            fh.write(_mutate(open(SRC).read(), old, new, occ))
        mlib = os.path.join(workdir, "libmutant.so")
        subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", mlib, msrc, "-lm"])
        env = dict(os.environ, DNNMG_ORACLE_LIB=mlib, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_fp8_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_paper_net_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_umesh_pins.py")],
                           env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
        return r.returncode, r.stdout[-2000:]
    except Exception as e:  # reported by the mutant's own test
        return e


@pytest.fixture(scope="module")
def mutant_results(tmp_path_factory):
    """Every mutant compiled and run once, in parallel (each is an
    independent compile and pytest process)."""
    base = tmp_path_factory.mktemp("mutants")
    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        futs = {name: ex.submit(_run_mutant, name, str(base / name)) for name in sorted(MUTATIONS)}
        return {name: f.result() for name, f in futs.items()}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, mutant_results):
    old, new, occ = MUTATIONS[name]
    assert open(SRC).read().count(old) > occ, "mutation anchor missing: %s" % name
    res = mutant_results[name]
    if isinstance(res, Exception):
        raise res
    code, out = res
    assert code != 0, "pins did not catch mutation %s:\n%s" % (name, out)
