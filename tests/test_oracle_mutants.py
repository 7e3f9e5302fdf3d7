"""Mistakes planted in the oracle, on the CPU: each entry below rewrites one
expression of ``oracle/grprec_oracle.c`` the way a plausible slip would (a
flipped sign, a wrong exponent, a transposed index, swapped operands), builds
that copy with the oracle's own flags, and runs the oracle's pin tests
against it.  Every planted mistake must make at least one pin fail; a
mistake that no pin catches would be a hole in what the pins prove.

The pins run in child processes (``GRPREC_ORACLE_LIB`` points the oracle
module at the mutated build), several at a time; the pristine oracle is not
touched.  Mistakes that cannot change any result (the Newton start, which
the solution does not depend on) are not planted."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "grprec_oracle.c")
PINS = ["tests/test_oracle_pieces.py", "tests/test_oracle_riemann.py", "tests/test_oracle_scheme.py",
        "tests/test_oracle_nl.py", "tests/test_oracle_source.py"]

# the pins' two slowest groups (a fine-grid integral identity and a
# convergence-rate run, ~20 s together) are left out of the planted runs to
# keep them short: every planted mistake is caught without them
SKIP = "not test_integral_conservation and not test_paper_euler_rates"

# (name, expression as written, the planted mistake)
MUTANTS = [
    ("rarefaction branch exponent (g-1)/g instead of (g-1)/(2g)",
     "*f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);",
     "*f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / g) - 1.0);"),
    ("shock branch B_K with (g+1)/(g-1)",
     "double bk = (g - 1.0) / (g + 1.0) * pk;",
     "double bk = (g + 1.0) / (g - 1.0) * pk;"),
    ("star velocity with f_L - f_R",
     "double u = 0.5 * (ul + ur) + 0.5 * (fr - fl);",
     "double u = 0.5 * (ul + ur) + 0.5 * (fl - fr);"),
    ("sampling side chosen by u* < 0",
     "  if (u >= 0.0) {\n    if (p <= pl) { /* left rarefaction */",
     "  if (u < 0.0) {\n    if (p <= pl) { /* left rarefaction */"),
    ("left shock star density ratio inverted",
     "W0[0] = rl * (pml + gm1 / gp1) / (pml * gm1 / gp1 + 1.0); W0[1] = u; W0[2] = p;",
     "W0[0] = rl * (pml * gm1 / gp1 + 1.0) / (pml + gm1 / gp1); W0[1] = u; W0[2] = p;"),
    ("Euler energy flux u E",
     "F[2] = u * (E + p);\n}",
     "F[2] = u * E;\n}"),
    ("pressure from E - m u",
     "double p = (cf->gamma - 1.0) * (E - 0.5 * mom * u);",
     "double p = (cf->gamma - 1.0) * (E - mom * u);"),
    ("time matrix with + integral",
     "K[b * n + l] = orc_lagr(n, s->g, b, 1.0) * orc_lagr(n, s->g, l, 1.0) - integral;",
     "K[b * n + l] = orc_lagr(n, s->g, b, 1.0) * orc_lagr(n, s->g, l, 1.0) + integral;"),
    ("space derivative matrix transposed",
     "acc += s->D[a][k] * F[(v * n + k) * n + l];",
     "acc += s->D[k][a] * F[(v * n + k) * n + l];"),
    ("implicit source with - z w",
     "if (b == l) K[b * n + l] += z * s->w[b];",
     "if (b == l) K[b * n + l] -= z * s->w[b];"),
    ("predictor start without K^-1 l(0)",
     "double val = s->Kinv_l0[b] * w[v * n + a] - nu * acc;",
     "double val = w[v * n + a] - nu * acc;"),
    ("end-of-step trace evaluated at t = 0",
     "for (int b = 0; b < n; ++b) qa1 += s->l1[b] * q[(v * n + a) * n + b];",
     "for (int b = 0; b < n; ++b) qa1 += s->l0[b] * q[(v * n + a) * n + b];"),
    ("left neighbour's mean over the right cell",
     "case 0: a = -1.5; b = -0.5; break;",
     "case 0: a = 0.5; b = 1.5; break;"),
    ("interface points -1/2 and +1/2 swapped",
     "static const double point[7] = {0.0, 0.0, 0.0, -0.5, 0.5, -1.5, 1.5};",
     "static const double point[7] = {0.0, 0.0, 0.0, 0.5, -0.5, -1.5, 1.5};"),
    ("Gauss-Legendre weights not halved on [0,1]",
     "w01[n - 1 - i] = 0.5 * w;",
     "w01[n - 1 - i] = w;"),
    ("S_max from u + c",
     "double si = fabs(W[1]) + c;",
     "double si = W[1] + c;"),
    ("update with + nu (F_R - F_L)",
     "q[vv * n + i] - nu * (Fb[vv * (n + 1) + i + 1] - Fb[vv * (n + 1) + i]) + dt * Si[vv * n + i];",
     "q[vv * n + i] + nu * (Fb[vv * (n + 1) + i + 1] - Fb[vv * (n + 1) + i]) + dt * Si[vv * n + i];"),
    ("source integral with - dt S",
     "q[vv * n + i] - nu * (Fb[vv * (n + 1) + i + 1] - Fb[vv * (n + 1) + i]) + dt * Si[vv * n + i];",
     "q[vv * n + i] - nu * (Fb[vv * (n + 1) + i + 1] - Fb[vv * (n + 1) + i]) - dt * Si[vv * n + i];"),
    ("oscillation indicator with dx^(2l-1)",
     "oi += dx * w[k] * d * d * pow(dx, 2 * l);",
     "oi += dx * w[k] * d * d * pow(dx, 2 * l - 1);"),
    ("GRPrecNL central weight with exponent r/2",
     "double wc = cf->nl_lambda_c / pow(cf->nl_eps + orc_oi_q(m, cc, dx, t->g5, t->w5), cf->nl_r);",
     "double wc = cf->nl_lambda_c / pow(cf->nl_eps + orc_oi_q(m, cc, dx, t->g5, t->w5), 0.5 * cf->nl_r);"),
    ("GRPrecNL left and right candidates swapped",
     "      cl[r] += ML[r * 7 + k] * d[k];\n      cr[r] += MR[r * 7 + k] * d[k];",
     "      cl[r] += MR[r * 7 + k] * d[k];\n      cr[r] += ML[r * 7 + k] * d[k];"),
    ("two-rarefaction exponent (g-1)/g",
     "double gm1 = g - 1.0, gp1 = g + 1.0, z = gm1 / (2.0 * g);",
     "double gm1 = g - 1.0, gp1 = g + 1.0, z = gm1 / g;"),
    ("right ghost cell holding the first cell's average",
     "GR[vv * (nn + 1) + b] = fac * q[vv * n + n - 1];",
     "GR[vv * (nn + 1) + b] = fac * q[vv * n + 0];"),
    ("V_{i+3/2} beyond a transmissive end read as the end interface's value",
     "vp = (i + 2 <= n) ? vvv[i + 2] : qv[n - 1];",
     "vp = (i + 2 <= n) ? vvv[i + 2] : vvv[n];"),
    ("right eigenvector of u - c with H + u c",
     "double col[3][3] = {{1.0, u - c, H - u * c}, {1.0, u, 0.5 * u * u}, {1.0, u + c, H + u * c}};",
     "double col[3][3] = {{1.0, u - c, H + u * c}, {1.0, u, 0.5 * u * u}, {1.0, u + c, H + u * c}};"),
    ("first-step datum from the left limit only",
     "      QR[vv] = vr[vv * nif + k];",
     "      QR[vv] = vl[vv * nif + k];"),
    ("Newton keeps a non-positive iterate's predecessor",
     "if (pn <= 0.0) pn = 0.5 * p;",
     "if (pn <= 0.0) pn = p;"),
    ("degree-3 least squares counting the right mean twice, not the left",
     "ls[nls++] = 2; ls[nls++] = 0; ls[nls++] = 3; ls[nls++] = 4;",
     "ls[nls++] = 2; ls[nls++] = 2; ls[nls++] = 3; ls[nls++] = 4;"),
    ("degree-2 candidates take the same-side interface value",
     "{{0, 1, 4}, {1, 2, 3}},", "{{0, 1, 3}, {1, 2, 4}},"),
    ("characteristic projection with R instead of R^-1",
     "w[k][j] += Lm[k * 3 + v] * d[v * 7 + j];", "w[k][j] += Rm[k * 3 + v] * d[v * 7 + j];"),
    ("projection back with R^-1",
     "coef[v * (m + 1) + r] += Rm[v * 3 + k] * cw[k][r];", "coef[v * (m + 1) + r] += Lm[v * 3 + k] * cw[k][r];"),
    ("advection interface state taken downwind",
     "Q0[0] = cf->lambda >= 0.0 ? QL[0] : QR[0];", "Q0[0] = cf->lambda >= 0.0 ? QR[0] : QL[0];"),
    ("flux time integral with equal weights",
     "for (int vv = 0; vv < nv; ++vv) Fbar[vv] += s.w[b] * F[vv];",
     "for (int vv = 0; vv < nv; ++vv) Fbar[vv] += F[vv] / nn;"),
    ("left end: ghost and cell traces swapped",
     "      tl = GL;\n      tr = TL;", "      tl = TL;\n      tr = GL;"),
    ("periodic interface between the wrong cells",
     "int cl = (k - 1 + n) % n, cr = k % n;", "int cl = k % n, cr = (k - 1 + n) % n;"),
    ("indicator quadrature on the shifted cell",
     "double xi = g[k] - 0.5; /* x = x_i + xi dx */", "double xi = g[k]; /* x = x_i + xi dx */"),
    ("side candidates' linear weight 2",
     "#define ORC_NL_LAMBDA_SIDE 1.0", "#define ORC_NL_LAMBDA_SIDE 2.0"),
    ("predictor data evaluated at g instead of g - 1/2",
     "w[vv * nn + a] = orc_poly(m, coef + vv * (m + 1), s.g[a] - 0.5);",
     "w[vv * nn + a] = orc_poly(m, coef + vv * (m + 1), s.g[a]);"),
    ("ghost states without the source's decay",
     "const double fac = kap == 0.0 ? 1.0 : (b < nn ? s.Kinv_l0[b] : gend);",
     "const double fac = 1.0;"),
    ("ghost end-of-step factor from the t = 0 basis values",
     "for (int b = 0; b < nn; ++b) gend += s.l1[b] * s.Kinv_l0[b];",
     "for (int b = 0; b < nn; ++b) gend += s.l0[b] * s.Kinv_l0[b];"),
    ("source integral without the time weights",
     "acc += s.w[a] * s.w[b] * (-kap * qh[(vv * nn + a) * nn + b]);",
     "acc += s.w[a] * (-kap * qh[(vv * nn + a) * nn + b]);"),
    ("two-rarefaction star velocity with the sound-speed changes swapped",
     "double u = 0.5 * (ul + ur) + ((csr - cr) - (csl - cl)) / gm1;",
     "double u = 0.5 * (ul + ur) + ((csl - cl) - (csr - cr)) / gm1;"),
    ("two-rarefaction left fan tested against u* + c*",
     "    } else if (u - csl < 0.0) {", "    } else if (u + csl < 0.0) {"),
    ("time step without the CFL number",
     "double d = cfl * dx / S;\n  if (d >= t_end - t) {", "double d = dx / S;\n  if (d >= t_end - t) {"),
    ("S_max dropping a NaN cell",
     "if (isnan(si) || isnan(s)) {", "if (isnan(s)) {"),
    ("primitive pressure without the kinetic half",
     "W[2] = (g - 1.0) * (Q[2] - 0.5 * Q[1] * W[1]);", "W[2] = (g - 1.0) * (Q[2] - Q[1] * W[1]);"),
    ("conserved energy with p (g - 1)",
     "Q[2] = W[2] / (g - 1.0) + 0.5 * W[0] * W[1] * W[1];", "Q[2] = W[2] * (g - 1.0) + 0.5 * W[0] * W[1] * W[1];"),
    ("Legendre recurrence with k + 1 in the second term",
     "double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;",
     "double pk = ((2.0 * k - 1.0) * x * p1 - (k + 1.0) * p0) / k;"),
    ("Lagrange derivative without the 1/(g_k - g_j) factor",
     "double term = 1.0 / (g[k] - g[j]);", "double term = 1.0;"),
    ("Lagrange basis with the node order reversed in the denominator",
     "if (j != k) v *= (x - g[j]) / (g[k] - g[j]);", "if (j != k) v *= (x - g[j]) / (g[j] - g[k]);"),
]


def _caught(args):
    k, (name, old, new), work = args
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant {k} ({name}): expression not found once in the oracle"
    path = os.path.join(work, f"m{k}.c")
    lib = os.path.join(work, f"libm{k}.so")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", lib, path, "-lm"])
    env = dict(os.environ, GRPREC_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", "-k", SKIP], cwd=ROOT, env=env, capture_output=True, text=True)
    # exit 1: some pin failed (caught); 0: every pin passed (survived)
    return k, name, r.returncode, r.stdout[-400:]


def test_every_planted_mistake_fails_a_pin():
    jobs = max(1, min(8, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 4))
    with tempfile.TemporaryDirectory() as work:
        with cf.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_caught, [(k, m, work) for k, m in enumerate(MUTANTS)]))
    survived = [(k, name, rc, tail) for k, name, rc, tail in results if rc != 1]
    assert not survived, "\n".join(f"mutant {k} ({name}): pytest exit {rc}\n{tail}" for k, name, rc, tail in survived)


def test_unplanted_oracle_passes_its_pins_in_the_same_harness():
    """The harness itself: the pristine source, built the same way and run
    the same way, passes (so a failure above is the planted mistake's)."""
    with tempfile.TemporaryDirectory() as work:
        lib = os.path.join(work, "libclean.so")
        subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", lib, SRC, "-lm"])
        env = dict(os.environ, GRPREC_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pieces.py",
                            "tests/test_oracle_riemann.py", "-x", "-q", "-p", "no:cacheprovider"],
                           cwd=ROOT, env=env, capture_output=True, text=True)
        assert r.returncode == 0, r.stdout[-800:]


# The float64 network reference (oracle/mlp.py): the same idea in-process.
# Each entry rewrites one line of a copy of the module; every test of
# tests/test_oracle_mlp.py is then run against the copy, and at least one
# must fail.
MLP_MUTANTS = [
    ("first weight block read transposed",
     "W1 = P[0:192].reshape(32, 6)", "W1 = P[0:192].reshape(6, 32).T"),
    ("forward standardises by multiplying with std",
     "def forward(P, x):\n    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)\n"
     "    z = (np.asarray(x, dtype=np.float64) - mean) / std",
     "def forward(P, x):\n    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)\n"
     "    z = (np.asarray(x, dtype=np.float64) - mean) * std"),
    ("forward adds the first bias after tanh",
     "def forward(P, x):\n    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)\n"
     "    z = (np.asarray(x, dtype=np.float64) - mean) / std\n    h1 = np.tanh(z @ W1.T + b1)",
     "def forward(P, x):\n    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)\n"
     "    z = (np.asarray(x, dtype=np.float64) - mean) / std\n    h1 = np.tanh(z @ W1.T) + b1"),
    ("pressure features in swapped slots",
     "np.log(WL[:, 2] / pbar),\n                  np.log(WR[:, 2] / pbar)",
     "np.log(WR[:, 2] / pbar),\n                  np.log(WL[:, 2] / pbar)"),
    ("sound speed without gamma",
     "cbar = np.sqrt(gamma * pbar / rbar)", "cbar = np.sqrt(pbar / rbar)"),
    ("backward through W2 transposed",
     "d1 = (d2 @ W2) * (1 - h1 * h1)         # upstream", "d1 = (d2 @ W2.T) * (1 - h1 * h1)         # upstream"),
    ("loss gradient without the factor 2",
     "dy = 2.0 * (y - t) / n", "dy = (y - t) / n"),
    ("Adam without the second-moment bias correction",
     "vh = v / (1 - b2 ** step)", "vh = v"),
]


def _mlp_tests():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_mlp_pins", os.path.join(ROOT, "tests", "test_oracle_mlp.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    tests = [getattr(mod, n) for n in dir(mod) if n.startswith("test_")]
    return mod, tests


@pytest.mark.parametrize("k", range(len(MLP_MUTANTS)))
def test_every_planted_network_mistake_fails_a_pin(k):
    import types
    name, old, new = MLP_MUTANTS[k]
    src = open(os.path.join(ROOT, "oracle", "mlp.py")).read()
    assert src.count(old) == 1, f"{name}: expression not found once in oracle/mlp.py"
    mutant = types.ModuleType("mlp_mutant")
    exec(compile(src.replace(old, new), "mlp_mutant", "exec"), mutant.__dict__)
    mod, tests = _mlp_tests()
    mod.mlp = mutant
    caught = []
    for t in tests:
        try:
            t()
        except Exception as e:  # a failed pin
            caught.append((t.__name__, type(e).__name__))
    assert caught, f"planted mistake '{name}' passed every network pin"


def test_unplanted_network_reference_passes_its_pins_in_the_same_harness():
    mod, tests = _mlp_tests()
    for t in tests:
        t()
