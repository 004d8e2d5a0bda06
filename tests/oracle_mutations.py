"""Mutation check of the oracle's pins (CPU only; test infrastructure).

It plants one plausible mistake at a time in a copy of an oracle component
(a flipped sign, a wrong index, a wrong coefficient or power, a changed step
rule) and runs that component's pin tests against the copy.  A mistake that
every pin lets pass marks a gap in the pins.  Two mistakes are expected to
pass: each changes a constant inside a rate formula where no property
independent of the formula depends on it (a slope of beta_m that rest does
not see, the functional form of the thin-filament relaxation rate); the GPU
models, written independently from the same formulas, catch such
transcription errors in the parity tests.

Not collected by pytest: it rebuilds the C oracle dozens of times (several
minutes).  Run it directly:

    python tests/oracle_mutations.py [core] [st57] [mlp] [emg]

Copies are built under tests/.mutants/ (ignored by git).  Exit status 1 if an
unexpected mistake passes every pin.
"""
import importlib.util
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
WORK = os.path.join(HERE, ".mutants")

# (name, text in the source, replacement)
CORE = [
    ("HH beta_m slope", "ab[1] = 4.0 * hh_exp(apx, -v / 18.0);", "ab[1] = 4.0 * hh_exp(apx, -v / 20.0);"),
    ("HH beta_h sign", "ab[3] = 1.0 / (hh_exp(apx, (30.0 - v) / 10.0) + 1.0);", "ab[3] = 1.0 / (hh_exp(apx, (v - 30.0) / 10.0) + 1.0);"),
    ("HH E_Na sign", "return gna * (V - HH_ENA)", "return gna * (V + HH_ENA)"),
    ("HH gate index", "dydt[2] = ab[2] * (1.0 - y[2]) - ab[3] * y[2];", "dydt[2] = ab[2] * (1.0 - y[2]) - ab[3] * y[1];"),
    ("HH gate sign", "dydt[1] = ab[0] * (1.0 - y[1]) - ab[1] * y[1];", "dydt[1] = ab[0] * (1.0 - y[1]) + ab[1] * y[1];"),
    ("Heun first order", "y[k] = y[k] + 0.5 * tau * (k1[k] + k2[k]);", "y[k] = y[k] + tau * k2[k];"),
    ("Heun stage half", "yt[k] = y[k] + tau * k1[k];", "yt[k] = y[k] + 0.5 * tau * k1[k];"),
    ("substeps floor", "int64_t n = (int64_t)ceil(span / dt - 1e-9);", "int64_t n = (int64_t)floor(span / dt + 1e-9);"),
    ("lumped end weight", "if (i == 0) { *wl = 0.0; *wr = 2.0; return; }", "if (i == 0) { *wl = 0.0; *wr = 1.0; return; }"),
    ("CN rhs weight swap", "b[i] = V[i] + expl * (wl * left - (wl + wr) * V[i] + wr * right);", "b[i] = V[i] + expl * (wr * left - (wl + wr) * V[i] + wl * right);"),
    ("CN explicit weight", "double impl = p->theta * lam, expl = (1.0 - p->theta) * lam;", "double impl = p->theta * lam, expl = p->theta * lam * 0.9;"),
    ("Thomas pivot", "x[i] = (b[i] - a[i] * x[i - 1]) / den;", "x[i] = (b[i] - a[i] * x[i - 1]) / d[i];"),
    ("CN coefficient", "double coef = p->sigma / (p->Am * p->Cm);", "double coef = p->sigma / p->Am;"),
    ('Strang order',
     '        reaction_range(p, S, yf, n, 0, n, I, 0.5 * dt);\n        diffusion_fiber(p, n, yf, dt, scratch);\n        reaction_range(p, S, yf, n, 0, n, I, 0.5 * dt);',
     '        reaction_range(p, S, yf, n, 0, n, I, 0.5 * dt);\n        reaction_range(p, S, yf, n, 0, n, I, 0.5 * dt);\n        diffusion_fiber(p, n, yf, dt, scratch);'),
    ("t_act reversed", "t_act[o + i] = t0 + dt * (p->v_th - v0) / (v1 - v0);", "t_act[o + i] = t0 + dt * (v1 - p->v_th) / (v1 - v0);"),
    ("t_act step shift", "double t0 = (double)step * dt;", "double t0 = (double)(step + 1) * dt;"),
    ("stim length", "return k < s->n_steps;", "return k <= s->n_steps;"),
    ("stim period", "if (s->period > 0) k = k % s->period;", "if (s->period > 0) k = k % (s->period + 1);"),
    ("sample index", "(step + 1) % sample_every == 0", "step % sample_every == 0"),
    ('vprev after prescribe',
     '      memcpy(vprev, yf, sizeof(double) * n);\n      fiber_prescribe(f, n, stim, n_stim, step, yf);',
     '      fiber_prescribe(f, n, stim, n_stim, step, yf);\n      memcpy(vprev, yf, sizeof(double) * n);'),
    ('stim half width',
     'for (int64_t j = (int64_t)s->node - s->half_width; j <= (int64_t)s->node + s->half_width; ++j)\n      if (j >= 0 && j < n) I[j] += s->amp;',
     'for (int64_t j = (int64_t)s->node - s->half_width; j < (int64_t)s->node + s->half_width; ++j)\n      if (j >= 0 && j < n) I[j] += s->amp;'),
    ("E_L constant", "#define HH_EL (HH_ER + 10.613)", "#define HH_EL (HH_ER + 10.0)"),
    ('adapt neighbor left',
     'if ((i > 0 && pt[i - 1] == OR_PT_ACTIVE) || (i + 1 < n && pt[i + 1] == OR_PT_ACTIVE))',
     'if ((i + 1 < n && pt[i + 1] == OR_PT_ACTIVE))'),
    ("adapt tolerance abs", "if (fabs(b - a) > tol * fabs(a)) moved[i] = 1;", "if (fabs(b - a) > tol) moved[i] = 1;"),
    ("adapt check only V", "    for (int k = 0; k < S; ++k) {\n      const double a = before", "    for (int k = 0; k < 1; ++k) {\n      const double a = before"),
    ("adapt no restim", "            if (j >= 0 && j < n) ptf[j] = OR_PT_ACTIVE;", "            if (j >= 0 && j < n && j == s->node) ptf[j] = OR_PT_ACTIVE;"),
    ("adapt first_on", "        first_on = stim[e].step_on;", "        first_on = stim[e].step_on + 1;"),
    ("adapt never diffuses", "          if (any) diffusion_fiber(p, n, yf, dt, scratch);\n          memcpy(before", "          if (any && 0) diffusion_fiber(p, n, yf, dt, scratch);\n          memcpy(before"),
    ('adapt check before',
     '          memcpy(before, yf, sizeof(double) * (size_t)S * n);\n          reaction_points(p, S, yf, n, ptf, I, 0.5 * dt);',
     '          reaction_points(p, S, yf, n, ptf, I, 0.5 * dt);\n          memcpy(before, yf, sizeof(double) * (size_t)S * n);'),
    ("exp* squarings", "  for (int i = 0; i < 10; ++i) u *= u;", "  for (int i = 0; i < 9; ++i) u *= u;"),
    ("log* break", "const double a = x < 2.0 ? 1.0 : (x < 6.0 ? 3.0 : 9.0);", "const double a = x < 2.0 ? 1.0 : (x < 5.0 ? 3.0 : 9.0);"),
    ("log* order", "  for (int k = 1; k <= 6; ++k) {", "  for (int k = 1; k <= 5; ++k) {"),
    ("log* series sign", "    s += (k % 2 ? p : -p) / (double)k;", "    s += p / (double)k;"),
    ("log* newton sign", "  y -= 1.0 - m / or_exp_star(y);", "  y += 1.0 - m / or_exp_star(y);"),
    ("log* scaling", "  return y + (double)k * log(2.0);", "  return y + (double)k * log(2.0) * 1.0001;"),
    ("x/expm1 series", "if (fabs(x) < 1e-4) return 1.0 - 0.5 * x + x * x / 12.0;", "if (fabs(x) < 1e-4) return 1.0 + 0.5 * x + x * x / 12.0;"),
    ("x/expm1 apx series", "if (fabs(x) < 1e-4) return 1.0 - a * x + (a * a - b) * x * x;", "if (fabs(x) < 1e-4) return 1.0 - 0.5 * x;"),
]
ST57 = [
    ("D index k_off", "- 0.115 * bT;", "- 0.115 * bP;"),
    ("D sign Jtr", "const double Jtr = 0.02 * (cs - cj);", "const double Jtr = 0.02 * (cj - cs);"),
    ("I sign gamma", "d[56] = (Fn - gam) / 5.0;", "d[56] = (Fn + gam) / 5.0;"),
    ("A sign Ic", "const double Ic = 0.2 * (V - Vt);", "const double Ic = 0.2 * (Vt - V);"),
    ("B sign coupling", "d[4] = (4.0 * 0.2 * (V - Vt)", "d[4] = (4.0 * 0.2 * (Vt - V)"),
    ("A sign ECl", "const double ECl = -KT * LOG(apx, 128.0 / Cli);", "const double ECl = KT * LOG(apx, 128.0 / Cli);"),
    ("E sign Ip in Na", "d[29] = -2e-5 * (INas + 4.0 * INat + 3.0 * Ip)", "d[29] = -2e-5 * (INas + 4.0 * INat - 3.0 * Ip)"),
    ("E sign Jp in Kt", "d[33] = 2e-3 * (IKt - 0.2 * Jp)", "d[33] = 2e-3 * (IKt + 0.2 * Jp)"),
    ("F index Jp", "const double Jp = J12;", "const double Jp = J23;"),
    ("C coefficient kb", "kb[i] = EXP(apx, -(Vt - Vi) / 25.0);", "kb[i] = EXP(apx, -(Vt - Vi) / 20.0);"),
    ("G formula rb", "const double rb = 0.3 / (1.0 + 5.0 * th);", "const double rb = 0.3 / (1.0 + 5.0 * th * th);"),
    ("H index R", "flux[0] = 1.5 * R[7] * X[0]", "flux[0] = 1.5 * R[6] * X[0]"),
    ("I index Fn", "const double Fn = 0.25 * X[4]", "const double Fn = 0.25 * X[3]"),
    ("A index gate", "d[1] = am * (1.0 - m) - bm * m;", "d[1] = am * (1.0 - m) - bm * h;"),
    ("B index gate", "const double INat = 12.0 * mt * mt * mt * ht", "const double INat = 12.0 * mt * mt * mt * h"),
    ("B sign EK", "const double EK = KT * LOG(apx, Kt / Ki);", "const double EK = KT * LOG(apx, Ki / Kt);"),
    ("E sign Cl", "d[31] = 2e-5 * (IClS + 4.0 * IClt)", "d[31] = -2e-5 * (IClS + 4.0 * IClt)"),
    ("D power Jup", "const double Jup = 4.0 * cplus * cplus / (1.0 + cplus * cplus);", "const double Jup = 4.0 * cplus / (1.0 + cplus * cplus);"),
    ("H index cycle back", "flux[7] = dtc * X[7] - 1e-4 * X[0];", "flux[7] = dtc * X[7] - 1e-4 * X[1];"),
    ("F sign back", "const double J30 = k4 * Q[3] - b4 * Q[0];", "const double J30 = k4 * Q[3] + b4 * Q[0];"),
]
MLP = [
    ("silu_grad", "return s * (1.0 + z * (1.0 - s))", "return s * (1.0 + z * s)"),
    ("output activation", "a = f(z) if i < len(params) - 1 else z", "a = f(z)"),
    ("loss scale", "dz = (O - T) / (B * n)", "dz = (O - T) / B"),
    ("bias grad axis", "gb = dz.sum(axis=0)", "gb = dz.mean(axis=0)"),
    ("backprop scale", "da = _mm(dz, W, bf16)", "da = _mm(dz, W, bf16) * 1.0001"),
    ("backprop activation", "dz = da * fg(zs[i - 1])", "dz = da * fg(acts[i])"),
    ("adam bias corr", "mh = m / (1 - b1 ** t)", "mh = m / (1 - b1 ** (t + 1))"),
    ("adam eps", "new.append(p - lr * mh / (np.sqrt(vh) + eps))", "new.append(p - lr * mh / np.sqrt(vh + eps))"),
    ("adam v update", "v = b2 * state[\"v\"][i][j] + (1 - b2) * g * g", "v = b2 * state[\"v\"][i][j] + (1 - b2) * np.abs(g)"),
    ("bf16 truncation", "u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = u & 0xFFFF0000"),
    ("bf16 ties up", "u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = (u + 0x8000) & 0xFFFF0000"),
    ("relu_grad at 0", "return (np.asarray(z) > 0.0).astype(np.float64)", "return (np.asarray(z) >= 0.0).astype(np.float64)"),
    ("unflatten order", "        W = vec[o:o + n_in * n_out].reshape(n_out, n_in)", "        W = vec[o:o + n_in * n_out].reshape(n_in, n_out).T"),
]
EMG = [
    ("stiffness corner", "    main[0] = main[-1] = 1.0\n", "    main[0] = main[-1] = 2.0\n"),
    ("mass diagonal", "    main = np.full(n, 4.0)\n", "    main = np.full(n, 2.0)\n"),
    ("mass corner", "    main[0] = main[-1] = 2.0\n    off = np.ones(n - 1)", "    main[0] = main[-1] = 4.0\n    off = np.ones(n - 1)"),
    ("kron order", "d[1] * sp.kron(Mz, sp.kron(Ky, Mx))", "d[1] * sp.kron(Mz, sp.kron(My, Kx))"),
    ("fiber axis", "d[2] * sp.kron(Kz, sp.kron(My, Mx))", "d[2] * sp.kron(Mz, sp.kron(My, Kx))"),
    ("intracellular tensor", "Ki = stiffness_3d(g, (0.0, 0.0, sigma_i))", "Ki = stiffness_3d(g, (sigma_i, 0.0, 0.0))"),
    ("total tensor", "Kt = stiffness_3d(g, (sigma_et, sigma_et, sigma_el + sigma_i))", "Kt = stiffness_3d(g, (sigma_et, sigma_et, sigma_el))"),
    ("rhs sign", "b = -(Ki @ V3)", "b = Ki @ V3"),
    ("prolong stride", "V3 = V[:, ::m][:, :nz]", "V3 = V[:, :nz]"),
    ("prolong layout", "return np.ascontiguousarray(V3.T).reshape(-1)", "return np.ascontiguousarray(V3).reshape(-1)"),
    ("mass scale", "* (h / 6.0)", "* (h / 3.0)"),
]
EXPECTED_SURVIVORS = {"HH beta_m slope", "G formula rb"}

GROUPS = {
    "core": ("fib_oracle.c", CORE, ["test_oracle_logstar.py", "test_oracle_hh.py", "test_oracle_strang.py",
                                    "test_oracle_diffusion.py", "test_oracle_tact.py",
                                    "test_oracle_adaptive.py"]),
    "st57": ("st57_oracle.c", ST57, ["test_oracle_st57.py"]),
    "mlp": ("mlp.py", MLP, ["test_oracle_mlp.py"]),
    "emg": ("emg.py", EMG, ["test_oracle_emg.py"]),
}

# pytest in a child process, with the oracle's C library or one of its
# Python modules replaced by the mutated copy
RUNNER = """
import sys, importlib.util
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
from oracle import oracle as O
kind, path = sys.argv[1], sys.argv[2]
if kind == "lib":
    O._LIB_PATH = path
    O._lib = None
else:
    import oracle
    spec = importlib.util.spec_from_file_location("oracle." + kind, path)
    m = importlib.util.module_from_spec(spec)
    sys.modules["oracle." + kind] = m
    spec.loader.exec_module(m)
    setattr(oracle, kind, m)
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *sys.argv[3:]]))
"""


def _build_lib(c_file, text):
    out = os.path.join(WORK, "mutant_" + c_file)
    with open(out, "w") as f:
        f.write(text)
    other = [os.path.join(ORACLE, s) for s in ("fib_oracle.c", "st57_oracle.c") if s != c_file]
    lib = os.path.join(WORK, "liboracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-o", lib, out, *other, "-lm"], check=True)
    return "lib", lib


def _write_module(py_file, text):
    out = os.path.join(WORK, "mutant_" + py_file)
    with open(out, "w") as f:
        f.write(text)
    return py_file[:-3], out


def main(groups):
    os.makedirs(WORK, exist_ok=True)
    runner = RUNNER.format(root=ROOT, tests=HERE)
    unexpected = []
    for g in groups:
        src_file, mutations, tests = GROUPS[g]
        src = open(os.path.join(ORACLE, src_file)).read()
        for name, a, b in mutations:
            if src.count(a) < 1:
                raise SystemExit(f"{g}: {name}: text not found in {src_file}")
            text = src.replace(a, b)
            kind, path = (_build_lib(src_file, text) if src_file.endswith(".c")
                          else _write_module(src_file, text))
            r = subprocess.run([sys.executable, "-c", runner, kind, path,
                                *[os.path.join(HERE, t) for t in tests]],
                               capture_output=True, text=True)
            failed = [l.split("::")[-1].split(" ")[0] for l in r.stdout.splitlines()
                      if l.startswith(("FAILED", "ERROR"))]
            if r.returncode:
                verdict = "caught by " + (failed[0] if failed else "an error")
            else:
                verdict = "passes every pin" + (" (expected)" if name in EXPECTED_SURVIVORS else "")
                if name not in EXPECTED_SURVIVORS:
                    unexpected.append(f"{g}: {name}")
            print(f"{g:5s} {name:24s} {verdict}", flush=True)
    if unexpected:
        print("unexpected survivors:", ", ".join(unexpected))
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:] or list(GROUPS)))
