"""The oracle's pins catch plausible slips (CPU only).

Each case copies oracle/ and tests/ into a temporary directory, plants one
mistake in the copied oracle source, builds it, and runs the pin suites
against it in a subprocess: at least one pin must fail. The committed oracle
is never modified.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "gyroscopic term without transpose": ("oracle.hpp",
        "m6_apply(m6_transpose(ad(V[i])), m6_apply(J, V[i]))", "m6_apply(ad(V[i]), m6_apply(J, V[i]))"),
    "gyroscopic term sign": ("oracle.hpp", "Fhat[i] = v6_sub(", "Fhat[i] = v6_add("),
    "parallel-axis sign": ("oracle.hpp",
        "J.a[i + 3][j + 3] = Ic[i][j] - m * cc;", "J.a[i + 3][j + 3] = Ic[i][j] + m * cc;"),
    "Ad off-diagonal sign": ("oracle.hpp", "      A.a[i][j + 3] = s;", "      A.a[i][j + 3] = -s;"),
    "ad off-diagonal sign": ("oracle.hpp", "A.a[i][j + 3] = Vv[i][j];", "A.a[i][j + 3] = -Vv[i][j];"),
    "Coriolis operands swapped": ("oracle.hpp",
        "m6_apply(X, dV[i - 1])), m6_apply(ad(Sqd), XV)", "m6_apply(X, dV[i - 1])), m6_apply(ad(XV), Sqd)"),
    "force recursion uses the wrong link transform": ("oracle.hpp",
        "? m6_identity<T>() : Ad(pose_inv(f[i + 1]));", "? m6_identity<T>() : Ad(pose_inv(f[i]));"),
    "exponential drops the [w]^2 v term": ("oracle.hpp",
        "T c = (k * t - sin(k * t)) / (k * k * k);", "T c = T(0);"),
    "quaternion off-diagonal sign": ("oracle.hpp",
        "g.R[0][1] = T(2) * (x * y - w * z);", "g.R[0][1] = T(2) * (x * y + w * z);"),
    "articulated inertia correction sign": ("oracle.hpp",
        "Jhat[i] = m6_add(ch.J(i), m6_sub(XtJX, corr));", "Jhat[i] = m6_add(ch.J(i), m6_add(XtJX, corr));"),
    "ABIA acceleration sign": ("oracle.hpp",
        "out[i] = chat[i] - v6_dot(Pi[i], lambda[i - 1]);", "out[i] = chat[i] + v6_dot(Pi[i], lambda[i - 1]);"),
    "ABIA backward uses tauhat_i": ("oracle.hpp",
        "v6_scale(Pi[i + 1], tauhat[i + 1]));", "v6_scale(Pi[i + 1], tauhat[i]));"),
    "explicit instead of semi-implicit Euler": ("oracle.hpp",
        "q[i] = q[i] + dt * qd[i];", "q[i] = q[i] + dt * (qd[i] - dt * qdd[i]);"),
    "bicomplex product cross-term sign": ("multicomplex.hpp",
        "x.a * y.b + x.b * y.a};", "x.a * y.b - x.b * y.a};"),
    "bicomplex sine: sin instead of cos in the i2 part": ("multicomplex.hpp",
        "return {std::sin(z.a) * std::cosh(z.b), std::cos(z.a) * std::sinh(z.b)};",
        "return {std::sin(z.a) * std::cosh(z.b), std::sin(z.a) * std::sinh(z.b)};"),
    "Hessian (q, qd) block seeds qdd": ("multicomplex.hpp",
        "(block == 1 || block == 2) ? 1 : 2;", "(block == 2) ? 1 : 2;"),
    "eq. (15) operand: velocity cross term sign": ("scan_form.py",
        "np.cross(a, s_v) + np.cross(s_w, b)", "np.cross(a, s_v) - np.cross(s_w, b)"),
    "eq. (15) operand: gyroscopic moment drops w x (I_O w)": ("scan_form.py",
        "np.cross(h, c) + wIw", "np.cross(h, c)"),
    "associative eq. (7): outer infinite direction not absorbed": ("scan_form.py",
        "WC1 = W @ C1f + np.outer(Bu, u1) / k", "WC1 = W @ C1f"),
    "associative eq. (7): projector on the wrong side": ("scan_form.py",
        "W = Binv - np.outer(Bu, u1 @ Q2 @ Binv) / k", "W = Binv - np.outer(Q2 @ Bu, u1 @ Binv) / k"),
    "gravity sign": ("__init__.py",
        "GRAVITY_ACC = np.array([0.0, 0.0, 9.81, 0.0, 0.0, 0.0])", "GRAVITY_ACC = np.array([0.0, 0.0, -9.81, 0.0, 0.0, 0.0])"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    fname, old, new = MUTANTS[name]
    dst = tmp_path / "m"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst / "oracle",
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), dst / "tests",
                    ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutations.py"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst / "pytest.ini")
    path = dst / "oracle" / fname
    src = path.read_text()
    assert src.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    path.write_text(src.replace(old, new))
    env = dict(os.environ, PYTHONPATH=f"{dst}{os.pathsep}{ROOT}")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle_pins.py", "tests/test_scan_form.py", "tests/test_oracle_grad.py",
                        "tests/test_oracle_hessian.py"],
                       cwd=dst, env=env, capture_output=True, text=True, timeout=600)
    assert "failed" in r.stdout, f"no pin failed for mutant '{name}':\n{r.stdout[-2000:]}\n{r.stderr[-2000:]}"
