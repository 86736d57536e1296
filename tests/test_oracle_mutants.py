"""The oracle's pins catch plausible mistakes.  Each case plants one mistake in a
copy of the oracle's C source (a dropped term, a wrong sign, a wrong index or
constant, a transposed operand), builds the copy on the CPU, and runs the
oracle's pin tests against it in a fresh process: at least one pin must fail.
The oracle itself is left untouched; only the copies are changed."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pabd_oracle.c")
HDR = os.path.join(ROOT, "oracle", "pabd_oracle.h")
PINS = ["tests/test_oracle_math.py", "tests/test_oracle_dynamics.py", "tests/test_oracle_contact.py",
        "tests/test_oracle_polynomial.py", "tests/test_oracle_augmented.py", "tests/test_oracle_driven.py",
        "tests/test_oracle_slider.py"]

# (name, text in the oracle, planted replacement); each text occurs once.
MUTANTS = [
    # prediction (Algorithm 1: explicit velocity and orientation update)
    ("gravity_dropped",
     "vs[k] = o->v[3 * b + k] + h * o->gravity[k];", "vs[k] = o->v[3 * b + k];"),
    ("quaternion_half_factor",
     "Qs[k] = Q[k] + 0.5 * h * dQ[k];", "Qs[k] = Q[k] + h * dQ[k];"),
    ("quaternion_product_order", "quat_mul(wq, Q, dQ);", "quat_mul(Q, wq, dQ);"),
    # quaternion read-off (Shepperd), the three non-trace branches
    ("shepperd_x_branch_sign", "q[3] = (R[7] - R[5]) / s;", "q[3] = (R[5] - R[7]) / s;"),
    ("shepperd_y_branch_sign", "q[3] = (R[2] - R[6]) / s;", "q[3] = (R[6] - R[2]) / s;"),
    ("shepperd_z_branch_index", "q[1] = (R[5] + R[7]) / s;\n  }\n}", "q[1] = (R[2] + R[7]) / s;\n  }\n}"),
    # generalised mass (Sec. 4.1.1)
    ("box_moment_axis",
     "Pi0[4] = *m * sy * sy / 12.0;", "Pi0[4] = *m * sx * sx / 12.0;"),
    ("sphere_moment_constant", "*m * r * r / 5.0", "*m * r * r / 3.0"),
    ("mass_block_index",
     "M[12 * (3 + 3 * blk + r) + 3 + 3 * blk + c] = Pi[3 * r + c];",
     "M[12 * (3 + 3 * blk + r) + 3 + 3 * blk + c] = Pi[3 * r + r];"),
    ("mass_block_diagonal_only",
     "M[12 * (3 + 3 * blk + r) + 3 + 3 * blk + c] = Pi[3 * r + c];",
     "M[12 * (3 + 3 * blk + r) + 3 + 3 * blk + c] = r == c ? Pi[3 * r + c] : 0.0;"),
    ("jacobian_transposed",
     "J[12 * r + 3 + 3 * r + k] = x[k];", "J[12 * r + 3 + 3 * k + r] = x[k];"),
    # global step (Sec. 4.2.1: implicit weight and explicit remainder)
    ("bond_h2_dropped_in_H",
     "/* implicit part: h^2 phi^+(d)/d J^T y_j with phi^+/d = kappa */\n"
     "        add_JTJ(xs, h2 * bd->kappa, H);",
     "/* implicit part: h^2 phi^+(d)/d J^T y_j with phi^+/d = kappa */\n"
     "        add_JTJ(xs, bd->kappa, H);"),
    ("spring_rest_sign",
     "add_JT(xs, nrm, h2 * (-bd->kappa * bd->rest), r);",
     "add_JT(xs, nrm, h2 * (bd->kappa * bd->rest), r);"),
    ("polynomial_binomial",
     "binom = binom * (double)(p - k) / (double)k;", "binom = binom * (double)(p - 1 - k) / (double)k;"),
    ("polynomial_split_sign",
     "pm -= binom * pow(d, (double)k) * lp;", "pm += binom * pow(d, (double)k) * lp;"),
    ("polynomial_weight_power",
     "pow(d, (double)(k - 1))", "pow(d, (double)k)"),
    # local step (Sec. 4.2.2)
    ("local_step_skipped",
     "pabd_oracle_polar(qh + 3, qnext + 12 * b + 3);",
     "memcpy(qnext + 12 * b + 3, qh + 3, 9 * sizeof(double));"),
    ("polar_reflection_kept",
     "double dsign = m3_det(UVt) < 0.0 ? -1.0 : 1.0;", "double dsign = 1.0;"),
    # residual
    ("residual_of_the_iterate",
     "num += m_norm2(o->mass[b], o->Pi + 9 * b, dq);",
     "num += m_norm2(o->mass[b], o->Pi + 9 * b, qk + 12 * b);"),
    # velocity recovery (Algorithm 1)
    ("recovery_gravity_twice",
     "o->v[3 * b + k] = (cnew[k] - o->c[3 * b + k]) / h;",
     "o->v[3 * b + k] = (cnew[k] - o->c[3 * b + k]) / h + h * o->gravity[k];"),
    ("recovery_product_transposed", "m3_mul(dA, Ainv, W);", "m3_mul(Ainv, dA, W);"),
    ("omega_sign",
     "o->w[3 * b + 0] = 0.5 * (W[7] - W[5]);", "o->w[3 * b + 0] = 0.5 * (W[5] - W[7]);"),
    # contacts and friction
    ("contact_gate_sign", "if (!(gap < 0.0)) {", "if (!(gap > 0.0)) {"),
    ("contact_kappa_h_power",
     "return o->kscale * m / (o->h * o->h);", "return o->kscale * m / o->h;"),
    ("friction_mu_dropped", "double s = b->mu * fn / ftn;", "double s = fn / ftn;"),
    ("contact_remainder_sign",
     "add_JT(xs, fe, side ? -h2 : h2, r);", "add_JT(xs, fe, side ? h2 : -h2, r);"),
    ("contact_end_swapped",
     "memcpy(yi, side ? yo : ys, sizeof yi);", "memcpy(yi, side ? ys : yo, sizeof yi);"),
    ("detection_margin_motion_dropped",
     "return o->margin + o->h * (v3_norm(o->v + 3 * b) + spin);", "return o->margin;"),
    ("box_face_axis_most_overlap",
     "if (best_axis < 0 || overlap < best) best = overlap, best_axis = ax;",
     "if (best_axis < 0 || overlap > best) best = overlap, best_axis = ax;"),
    ("box_face_normal_sign",
     "double sgn = v3_dot(axis, towards) >= 0.0 ? 1.0 : -1.0;",
     "double sgn = v3_dot(axis, towards) >= 0.0 ? -1.0 : 1.0;"),
    ("box_lateral_extent_ignored", "if (!lateral) continue;", "if (!lateral && 0) continue;"),
    ("sphere_box_gap_sign", "gap = dist - r;", "gap = dist + r;"),
    ("sphere_box_inside_gap", "gap = -best - r;", "gap = -best + r;"),
    ("sphere_box_point_side", "pw[k] = -r * nw[k];", "pw[k] = r * nw[k];"),
    ("sphere_box_inside_normal_side",
     "double sgn = pl[ks] >= 0.0 ? 1.0 : -1.0;", "double sgn = pl[ks] >= 0.0 ? -1.0 : 1.0;"),
    # driven joint (reading of Sec. 5.3.3)
    ("driven_amplitude_sign",
     "double th = dr[9] + dr[10] * sin(2.0 * M_PI * dr[11] * t + dr[12]);",
     "double th = dr[9] - dr[10] * sin(2.0 * M_PI * dr[11] * t + dr[12]);"),
    ("driven_turn_sense", "rotate_about(dr, th, rel, rot);", "rotate_about(dr, -th, rel, rot);"),
    # slider bond (reading of Sec. 5.1's slider joints)
    ("slider_foot_at_the_anchor",
     "const double t = v3_dot(dv, g) / v3_dot(g, g);", "const double t = 0.0 * v3_dot(dv, g);"),
    ("slider_foot_direction_sign",
     "xf[k] = b->xj[k] + t * b->axis[k];", "xf[k] = b->xj[k] - t * b->axis[k];"),
    ("slider_axis_in_world_frame",
     "    m3_vec(q + 12 * b->j + 3, b->axis, g);", "    memcpy(g, b->axis, sizeof g);"),
    ("slider_line_side_arm_at_the_anchor",
     "add_JTJ(xf, h2 * bd->kappa, H);\n            add_JT(xf, yi, h2 * bd->kappa, r);",
     "add_JTJ(bd->xj, h2 * bd->kappa, H);\n            add_JT(bd->xj, yi, h2 * bd->kappa, r);"),
    ("slider_line_side_drawn_to_its_foot",
     "add_JT(xf, yi, h2 * bd->kappa, r);", "add_JT(xf, yf, h2 * bd->kappa, r);"),
    ("driven_time_at_step_start",
     "const double t = o->t0 + (double)(o->steps_done + 1) * h;",
     "const double t = o->t0 + (double)o->steps_done * h;"),
    # augmented bonds (Sec. 5.2.2)
    ("augmented_warm_start_floor_dropped",
     "b->al_kappa = fmax(o->al_gamma * b->al_kappa, b->kappa);",
     "b->al_kappa = o->al_gamma * b->al_kappa;"),
    ("augmented_lambda_term_dropped",
     "bd->al_lambda = bd->al_kappa * al_C[e] + bd->al_lambda;",
     "bd->al_lambda = bd->al_kappa * al_C[e];"),
    ("augmented_kappa_abs_dropped",
     "bd->al_kappa = bd->al_kappa + o->al_beta * fabs(al_C[e]);",
     "bd->al_kappa = bd->al_kappa + o->al_beta * al_C[e];"),
    ("augmented_warm_start_alpha_dropped",
     "b->al_lambda = o->al_alpha * o->al_gamma * b->al_lambda;",
     "b->al_lambda = o->al_gamma * b->al_lambda;"),
    ("augmented_warm_start_gamma_dropped",
     "b->al_lambda = o->al_alpha * o->al_gamma * b->al_lambda;",
     "b->al_lambda = o->al_alpha * b->al_lambda;"),
    ("augmented_split_side",
     "if (phim > 0.0 && d > 1e-12) {", "if (phim < 0.0 && d > 1e-12) {"),
]


def test_every_planted_text_occurs_once():
    src = open(SRC).read()
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, name
        assert old != new, name


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed to build the copies")
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1
    (tmp_path / "pabd_oracle.c").write_text(src.replace(old, new))
    shutil.copy(HDR, tmp_path / "pabd_oracle.h")
    lib = tmp_path / "libpabd_oracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib),
                           str(tmp_path / "pabd_oracle.c"), "-lm"])
    env = dict(os.environ, PABD_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # 0: every pin passed (the mistake went unnoticed); 5: nothing collected
    assert r.returncode not in (0, 5), f"{name} passed every pin:\n{r.stdout[-1500:]}"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed to build the copy")
def test_pins_pass_on_an_oracle_built_with_undefined_behaviour_checks(tmp_path):
    """The oracle's host code under the undefined-behaviour sanitizer (signed
    overflow, invalid shifts, misaligned or null access, out-of-range array
    indices where the bound is known), in trap mode, so that no sanitizer runtime
    is needed: any such event ends the process, and every pin must still pass."""
    lib = tmp_path / "libpabd_oracle_ubsan.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=undefined", "-fsanitize=bounds-strict",
                           "-fsanitize-undefined-trap-on-error", "-o", str(lib), SRC, "-lm"])
    env = dict(os.environ, PABD_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *PINS, "tests/test_oracle_checkpoint.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-1000:]
