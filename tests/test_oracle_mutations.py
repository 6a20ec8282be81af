"""The pins are strong enough: each plausible mistake planted in a copy of the
oracle (a flipped sign, a dropped term, a transposed operand, a wrong index)
makes at least one pin fail.  Mutants are built into a temporary directory on
the CPU; the repository's oracle is never modified.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, original text, mutated text, pin files expected to catch it)
PINS = "tests/test_oracle_pins.py"
GRADS = "tests/test_oracle_gradients.py"
TEMPORAL = "tests/test_oracle_temporal.py"
MARCH = "tests/test_oracle_raymarch.py"
NET = "tests/test_oracle_netinputs.py"
EWA = "tests/test_oracle_ewa.py"
EXACT = "tests/test_relproj_exact_cpu.py"
MUTANTS = [
    ("tie_not_to_even", "return (lb & 1u) == 0 ? below : above;", "return above;", EXACT),
    ("tie_rule_dropped", "if (qabs(x - half) <= 0x1p-100Q * m) {", "if (0) {", EXACT),
    ("sign_of_s", "const real s = (real)Dk - X[2];\n        if (s < -tau) continue; /* occluded",
     "const real s = X[2] - (real)Dk;\n        if (s < -tau) continue; /* occluded", PINS),
    ("no_occlusion_cut", "if (s < -tau) continue; /* occluded in view k */", "", PINS),
    ("transposed_rotation", "RaT[3 * r + k] = a->R[3 * k + r];",
     "RaT[3 * r + k] = a->R[3 * r + k];", PINS),
    ("residue_snap_too_coarse", "const quad tiny = 0x1p-50Q;", "const quad tiny = 0x1p-3Q;", PINS),
    ("pixel_corner_not_centre",
     "ray_of(Hk[k], (real)x + (real)0.5, (real)y + (real)0.5, h[k]);",
     "ray_of(Hk[k], (real)x, (real)y + (real)0.5, h[k]);", PINS),
    ("window_divisor_dropped", "RSQRT(nu / n2)", "RSQRT(nu)", PINS),
    ("hole_neighbour_free", "          } else {\n            term = tw2;",
     "          } else {\n            term = 0;", PINS),
    ("no_decay", "RMIN((decay * W_prev[o]) * m, cap)", "RMIN((W_prev[o]) * m, cap)", PINS),
    ("no_cap", "RMIN((decay * W_prev[o]) * m, cap)", "((decay * W_prev[o]) * m)", PINS),
    ("unnormalised_F", "F[o] = (Wn > 0) ? RFMA(wp, Fp, S) / Wn : (real)0;",
     "F[o] = (Wn > 0) ? RFMA(wp, Fp, S) : (real)0;", PINS),
    ("no_clamp", "const real cval = RMIN(s, tau);\n        const real w = conf[ns * k + q];\n        S",
     "const real cval = s;\n        const real w = conf[ns * k + q];\n        S", PINS),
    ("crossing_strict", "f[d] > 0 && f[d + 1] <= 0", "f[d] > 0 && f[d + 1] < 0", PINS),
    ("interpolation_flipped", "depth[n] = zb[d] + (zb[d + 1] - zb[d]) * frac;",
     "depth[n] = zb[d] + (zb[d + 1] - zb[d]) * (1 - frac);", PINS),
    ("bin_step", "const real du = (un - uf) / (real)(D - 1);",
     "const real du = (un - uf) / (real)(D);", PINS),
    ("truncation_width", "((real)p->trunc * du) * (z[d] * z[d])", "((real)p->trunc * du) * (z[d])",
     PINS),
    ("coverage_radius", "g->R2 = RMIN((real)2 * g->s2, rmax2);", "g->R2 = RMIN(g->s2, rmax2);", PINS),
    ("no_band", "if (!(g.z <= zwin[p] * band)) continue;", "if (!(g.z <= zwin[p])) continue;", PINS),
    ("gaussian_scale", "const real G = REXP(((real)-0.5 * d2) / g.s2);\n            nrm[p]",
     "const real G = REXP(((real)-1 * d2) / g.s2);\n            nrm[p]", PINS),
    ("alpha_complement", "out_alpha[o] = (real)1 - prod[p];", "out_alpha[o] = prod[p];", PINS),
    ("focal_ratio_dropped",
     "(real)((double)sp->sigma_px * (double)tgt->fx / (double)src[k].fx);\n    const float *dk = depth + ns * k;\n    const uint8_t *ck = rgb + ns * 3 * k;\n    real *prgb",
     "(real)((double)sp->sigma_px);\n    const float *dk = depth + ns * k;\n    const uint8_t *ck = rgb + ns * 3 * k;\n    real *prgb",
     PINS),
    ("grad_clamp_ignored", "if (s < tau) {\n          g_depth_in[ns * k + q] += gF[e] * w / Wn;",
     "if (1) {\n          g_depth_in[ns * k + q] += gF[e] * w / Wn;", GRADS),
    ("grad_neighbour_term", "g_depth_in[ns * k + n] -= gnu * (real)2 * dd;", "", GRADS),
    ("grad_alpha_term", "dLdG += g_alpha[o] * others;", "", GRADS),
    ("grad_footprint_term", "d2 * dsdD / (sig * g.s2)", "0", GRADS),
    ("mask_no_beta", "RMIN(t + (real)beta, (real)1)", "RMIN(t, (real)1)", TEMPORAL),
    ("mask_lambda_multiplies", "const real t = dI / (real)lambda_t;",
     "const real t = dI * (real)lambda_t;", TEMPORAL),
    ("mask_unclamped", "RMIN(t + (real)beta, (real)1)", "(t + (real)beta)", TEMPORAL),
    ("mask_no_pool", "pool[(size_t)b * Wq + a] = m;",
     "pool[(size_t)b * Wq + a] = low[(size_t)b * Wq + a];", TEMPORAL),
    ("mask_corner_sampling", "real x = ((real)i + (real)0.5) / (real)factor - (real)0.5;",
     "real x = (real)i / (real)factor;", TEMPORAL),
    ("mask_weights_swapped", "const real top = m00 + fx * (m10 - m00);",
     "const real top = m00 + fy * (m10 - m00);", TEMPORAL),
    ("mask_box_count", "const real dI = (real)d / (real)(765 * n);",
     "const real dI = (real)d / (real)(765 * factor * factor);", TEMPORAL),
    ("filter_weights_swapped", "out[p] = RFMA(mask[p], (real)D, a * prev[p]);",
     "out[p] = RFMA(a, (real)D, mask[p] * prev[p]);", TEMPORAL),
    ("filter_hole_kept", "    if (!depth_ok(D)) {\n      out[p] = 0;",
     "    if (!depth_ok(D) && 0) {\n      out[p] = 0;", TEMPORAL),
    ("mask_splat_unnormalised", "msum[p] / nrm[p];", "msum[p];", TEMPORAL),
    ("mask_max_not_max", "if (out_mask_max && m > out_mask_max[p]) out_mask_max[p] = m;",
     "if (out_mask_max) out_mask_max[p] = m;", TEMPORAL),
    ("march_full_step", "z = z + RMAX((real)0.8 * s, smin);", "z = z + RMAX(s * (real)1.6, smin);",
     MARCH),
    ("march_no_min_step", "z = z + RMAX((real)0.8 * s, smin);", "z = z + (real)0.8 * s;", MARCH),
    ("march_two_bisections", "for (int it = 0; it < 3; ++it) {", "for (int it = 0; it < 2; ++it) {",
     MARCH),
    ("march_bisection_flipped", "        if (f.Wt > 0 && f.S / f.Wt > 0)\n          a = mid;",
     "        if (f.Wt > 0 && f.S / f.Wt > 0)\n          b = mid;", MARCH),
    ("march_bracket_end", "      dep = a + (b - a) * (real)0.5;", "      dep = b;", MARCH),
    ("march_temporal_sign", "    const real s = Dp - z;", "    const real s = z - Dp;", MARCH),
    ("march_temporal_no_cap", "wtmp = RMIN((decay * acc[n]) * m, cap);", "wtmp = (decay * acc[n]) * m;",
     MARCH),
    ("march_acc_without_tmp", "      an = wtmp + f.Wo;", "      an = f.Wo;", MARCH),
    ("march_unnormalised", "        const real s = f.S / f.Wt;", "        const real s = f.S;", MARCH),
    ("net_normal_unoriented", "            if (dot3(nrm, tc) < 0)", "            if (0)", NET),
    ("net_cross_order", "tx[0] * ty[1] - tx[1] * ty[0]}", "tx[1] * ty[0] - tx[0] * ty[1]}", NET),
    ("net_ray_from_target", "real r3[3] = {X[0] - Cs[k][0], X[1] - Cs[k][1], X[2] - Cs[k][2]};",
     "real r3[3] = {X[0] - C[0], X[1] - C[1], X[2] - C[2]};", NET),
    ("net_one_sided_only", "tx[r] = v[0] && v[1] ? P[1][r] - P[0][r]", "tx[r] = 0 ? P[1][r] - P[0][r]",
     NET),
    ("net_axis_row", "ax += (double)src[k].R[6 + r] * (double)tgt->R[6 + r];",
     "ax += (double)src[k].R[3 + r] * (double)tgt->R[6 + r];", NET),
    ("blend_no_alpha", "const real aw = (real)alpha[k * n + p] * (real)w[k * n + p];",
     "const real aw = (real)w[k * n + p];", NET),
    ("blend_bg_swapped", "RFMA(wb, (real)rgb_bg[c * n + p], ((real)1 - wb) * fg);",
     "RFMA((real)1 - wb, (real)rgb_bg[c * n + p], wb * fg);", NET),
    ("exp_poly_coefficient", "p = fmaf(p, r, 1.0f / 24.0f);", "p = fmaf(p, r, 1.0f / 20.0f);",
     EWA),
    ("exp_reduction_tail", "r = fmaf(-n, 1.42860677e-6f, r);", "", EWA),
    ("ewa_no_lowpass_x", "const real sxx = s2 * ((real)1 + a * a) + lp;",
     "const real sxx = s2 * ((real)1 + a * a);", EWA),
    ("ewa_jacobian_wrong_axis", "const real sxx = s2 * ((real)1 + a * a) + lp;",
     "const real sxx = s2 * ((real)1 + b * b) + lp;", EWA),
    ("ewa_cross_sign", "g[q].Bn = sxy / det;", "g[q].Bn = -sxy / det;", EWA),
    ("ewa_conic_transposed", "g[q].Ah = ((real)-0.5 * syy) / det;",
     "g[q].Ah = ((real)-0.5 * sxx) / det;", EWA),
    ("ewa_focal_ratio_dropped",
     "(real)((double)sp->sigma_px * (double)tgt->fx / (double)src[k].fx);\n    const float *dk = depth + ns * k;\n    const uint8_t *ck = rgb + ns * 3 * k;\n    orc_ewa_entry",
     "(real)((double)sp->sigma_px);\n    const float *dk = depth + ns * k;\n    const uint8_t *ck = rgb + ns * 3 * k;\n    orc_ewa_entry",
     EWA),
    ("ewa_no_alpha_cap", "const real al = RMIN((real)0.99, G);", "const real al = G;", EWA),
    ("ewa_no_alpha_floor", "if (al < amin) continue;", "", EWA),
    ("ewa_stop_skips", "if (tt < (real)1e-4) break;", "if (tt < (real)1e-4) continue;", EWA),
    ("ewa_no_stop", "if (tt < (real)1e-4) break;", "", EWA),
    ("ewa_back_to_front", "return a < b ? -1 : (a > b ? 1 : 0);",
     "return a < b ? 1 : (a > b ? -1 : 0);", EWA),
    ("ewa_ties_reversed", "g[q].key = ((uint64_t)f32_bits((float)X[2]) << 32) | (uint32_t)q;",
     "g[q].key = ((uint64_t)f32_bits((float)X[2]) << 32) | (uint32_t)(ns - 1 - q);", EWA),
    ("ewa_depth_unnormalised", "T < 1 ? zs / ((real)1 - T) : (real)0;", "T < 1 ? zs : (real)0;",
     EWA),
    ("ewa_weight_after_update", "const real w = al * T;", "const real w = al * tt;", EWA),
    ("ewa_no_clip", "if (!(RABS(dx) <= rmax && RABS(dy) <= rmax)) continue;", "", EWA),
    ("ewa_corner_pixels",
     "const real px = (real)(int)(p % Wt) + (real)0.5, py = (real)(int)(p / Wt) + (real)0.5;",
     "const real px = (real)(int)(p % Wt), py = (real)(int)(p / Wt) + (real)0.5;", EWA),
]


def _run_mutant(name, orig, mut, pins):
    """Build a copy of the oracle with one mistake planted and run the pins
    that should catch it; returns (pytest exit code, output tail)."""
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    if src.count(orig) < 1:
        return -1, "mutation site not found"
    tmp = tempfile.mkdtemp(prefix=f"mut_{name}_")
    try:
        root = os.path.join(tmp, "root")
        shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(root, "oracle"),
                        ignore=shutil.ignore_patterns("*.so", "*.tmp", "__pycache__"))
        with open(os.path.join(root, "oracle", "oracle.c"), "w") as f:
            f.write(src.replace(orig, mut, 1))
        subprocess.run([sys.executable, os.path.join(root, "oracle", "build.py")], check=True,
                       capture_output=True)
        os.symlink(os.path.join(ROOT, "scenes"), os.path.join(root, "scenes"))
        shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(root, "tests"),
                        ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutations.py"))
        env = dict(os.environ, PYTHONPATH=root, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            "-m", "not gpu", pins], cwd=root, env=env, capture_output=True,
                           text=True)
        return r.returncode, r.stdout[-2000:]
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.fixture(scope="module")
def mutant_results():
    """Every mutant built and checked once, several at a time."""
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        futs = {m[0]: ex.submit(_run_mutant, *m) for m in MUTANTS}
        return {k: f.result() for k, f in futs.items()}


@pytest.mark.slow
@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_mutant_is_caught(name, mutant_results):
    rc, out = mutant_results[name]
    assert rc != -1, "mutation site not found"
    assert rc == 1, f"mutant {name} survived:\n{out}"
