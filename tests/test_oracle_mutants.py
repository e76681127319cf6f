"""The oracle's pins catch plausible mistakes.

Each mutant plants one mistake of the kind that slips into such code (a
dropped term, a wrong sign, factor, constant or index, swapped operands) into
a copy of the oracle's source, builds it on the CPU, and runs the pin suite
(tests/test_oracle_*.py) against it through VSH_ORACLE_LIB.  Every mutant
must fail at least one pin; the committed oracle itself passes them all.

Known blind spots: the overestimate's z range narrowed inside the physical
limits z(1 - z) = t_C / Q^2 (say by a factor 1.5 in t_C / Q^2) loses only a
sliver where the (1 - y) factor already suppresses the density: 2.5% of the
emission probability at sqrt(s) = 6 GeV, t_C = 4 GeV^2, about 3 standard
deviations of the near-threshold pin.  A wider range only costs efficiency
(the veto's y < 1 trims it to the true phase space).  For the same reason
the massive z range taken without the spectator mass (a wider range) only
costs efficiency.  The massive map's clamp of the Kallen function at zero is
no mutant either: where it would act, the map's p_k coefficient (which
divides by that function) has no finite value anyway, and the phase-space
factor gives that edge no weight.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vsh_oracle.c")
PINS = ["tests/test_oracle_rng.py", "tests/test_oracle_physics.py", "tests/test_oracle_shower.py",
        "tests/test_oracle_observables.py", "tests/test_oracle_massive.py", "tests/test_oracle_validation.py",
        "tests/test_oracle_isr.py"]

# (name, text in vsh_oracle.c, replacement)
MUTANTS = [
    ("philox multiplier", "(uint64_t)0xD2511F53u * (uint64_t)x0", "(uint64_t)0xD2511F55u * (uint64_t)x0"),
    ("philox key schedule", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;"),
    ("alpha_s beta0 sign of n_f", "(33.0 - 2.0 * NF)", "(33.0 + 2.0 * NF)"),
    ("alpha_s running direction", "1.0 + ASMZ * b0 * log", "1.0 - ASMZ * b0 * log"),
    ("q->qg dropped (1+z)", "(1.0 - z * (1.0 - y)) - (1.0 + z));", "(1.0 - z * (1.0 - y)) - 1.0);"),
    ("g->gg z(1-z) doubled", "- 2.0 + z * (1.0 - z));", "- 2.0 + 2.0 * z * (1.0 - z));"),
    ("g->qqbar 2z(1-z) halved", "(1.0 - 2.0 * z * (1.0 - z));", "(1.0 - z * (1.0 - z));"),
    ("q overestimate factor", "return 2.0 * CF / (1.0 - z);", "return CF / (1.0 - z);"),
    ("q overestimate integral factor", "return 2.0 * CF * log((1.0 - zm) / (1.0 - zp));",
     "return CF * log((1.0 - zm) / (1.0 - zp));"),
    ("z inverse with swapped limits", "pow((1.0 - zp) / (1.0 - zm), u)", "pow((1.0 - zm) / (1.0 - zp), u)"),
    ("ME without Z/gamma interference", "*B = 4.0 * qe * qf * ae * af * chi1", "*B = 0.0 * qe * qf * ae * af * chi1"),
    ("ME |Z|^2 coupling sign", "(af * af + vf * vf) * chi2", "(af * af - vf * vf) * chi2"),
    ("CS map: z and 1-z swapped for i", "out_i[m] = z * pi[m] + (1.0 - z) * y * pk[m] + kperp;",
     "out_i[m] = (1.0 - z) * pi[m] + z * y * pk[m] + kperp;"),
    ("CS map: k_perp sign of j", "out_j[m] = (1.0 - z) * pi[m] + z * y * pk[m] - kperp;",
     "out_j[m] = (1.0 - z) * pi[m] + z * y * pk[m] + kperp;"),
    ("CS map: spectator recoil", "out_k[m] = (1.0 - y) * pk[m];", "out_k[m] = (1.0 - y * z) * pk[m];"),
    ("CS map: azimuth basis", "double kperp = kt * (cphi * n1[m] + sphi * n2[m]);",
     "double kperp = kt * (cphi * n1[m] + sphi * n1[m]);"),
    ("trial scale exponent", "double t_try = t * pow(u, 1.0 / c);", "double t_try = t * pow(u, c);"),
    ("trial coefficient 2 pi", "double c = asmax / (2.0 * OR_PI) * or_kernel_integral(K, zm, zp);",
     "double c = asmax / OR_PI * or_kernel_integral(K, zm, zp);"),
    ("dipole-end threshold at the running scale", "if (!(q2 > 4.0 * tcut)) continue;",
     "if (!(q2 > 4.0 * t)) continue;"),
    ("veto without the (1-y) measure", "or_kernel_value(wK, z, y) * (1.0 - y) /", "or_kernel_value(wK, z, y) /"),
    ("veto alpha_s at the cutoff", "prob = or_alpha_s(t) / asmax * or_kernel_value",
     "prob = or_alpha_s(tcut) / asmax * or_kernel_value"),
    ("uniform for the veto from the z words", "double uv = or_uniform(a[2], a[3]);", "double uv = or_uniform(a[0], a[1]);"),
    ("colour line not moved to the emitter", "        jacol = m;\n        col[wi] = m;",
     "        jacol = m;\n        col[wi] = col[wi];"),
    ("g->qqbar flavour sign", "        pid[wi] = -f;\n", "        pid[wi] = f;\n"),
    ("thrust: sign of the out-of-plane partons", "double sg = d > 0.0 ? 1.0 : -1.0;", "double sg = d > 0.0 ? 1.0 : 1.0;"),
    ("thrust: in-plane sign choices", "w[m] = v[m] + sgn[c][0] * pi[m] + sgn[c][1] * pj[m];",
     "w[m] = v[m] + pi[m] + pj[m];"),
    ("Durham: max instead of min energy", "double emin = jet[a][0] < jet[b][0] ? jet[a][0] : jet[b][0];",
     "double emin = jet[a][0] > jet[b][0] ? jet[a][0] : jet[b][0];"),
    ("Durham: merge without the energy", "for (int c = 0; c < 4; ++c) jet[ba][c] += jet[bb][c];",
     "for (int c = 1; c < 4; ++c) jet[ba][c] += jet[bb][c];"),
    ("C-parameter prefactor", "double c = 1.5 * (sum * sum - dbl) / (sum * sum);",
     "double c = 1.0 * (sum * sum - dbl) / (sum * sum);"),
    ("wide broadening as the minimum", "*b_w = bp > bm ? bp : bm;", "*b_w = bp < bm ? bp : bm;"),
    ("tail cut one cycle late", "if (max_cycles > 0 && cycle >= (uint32_t)max_cycles) {",
     "if (max_cycles > 0 && cycle > (uint32_t)max_cycles) {"),
    ("weighted veto: rejections keep a positive weight", "wgt *= accept ? 2.0 * prob - 1.0 : -(2.0 * prob - 1.0);",
     "wgt *= accept ? 2.0 * prob - 1.0 : (2.0 * prob - 1.0);"),
    ("weighted veto: always accept above the trial density", "accept = uv < e;", "accept = 1;"),
    ("weighted veto: acceptance one half", "double e = prob / (2.0 * prob - 1.0);", "double e = 0.5;"),
    ("massive flux inverted", "return (Q2 - mi * mi - mj * mj - mk * mk) / sqrt(kallen(Q2, mij * mij, mk * mk));",
     "return sqrt(kallen(Q2, mij * mij, mk * mk)) / (Q2 - mi * mi - mj * mj - mk * mk);"),
    ("massive Q -> Q g mass term halved", "- 2.0 * mi * mi / (y * qb2));", "- mi * mi / (y * qb2));"),
    ("massive Jacobian dy/y taken as dt/t", "(t / (t + cz))", "(1.0)"),
    ("massive map without the spectator rescaling",
     "double scale = sqrt((lam > 0.0 ? lam : 0.0) / kallen(Q2, mij * mij, mk * mk));", "double scale = 1.0;"),
    ("massive map: sign of the p_k coefficient", "double bb = (mi2 - mj2 - (2.0 * z - 1.0) * s)",
     "double bb = (mi2 - mj2 + (2.0 * z - 1.0) * s)"),
    ("massive ME: axial current with the vector threshold", "aa * b2 * (1.0 + c * c)",
     "aa * (2.0 - b2 * (1.0 - c * c))"),
    ("massive ME: phase-space beta dropped", "wt = (double)n_open * beta * or_me2_massive(",
     "wt = (double)n_open * or_me2_massive("),
    ("closed flavours produced", "if (!mass || 4.0 * mass[f] * mass[f] < s) open[n_open++] = f;",
     "open[n_open++] = f;"),
    ("mass shells ignored in validation", "if (fabs(mdot(&p[4 * a], &p[4 * a]) - m * m) > 1e-10 * ecm * ecm)",
     "if (fabs(mdot(&p[4 * a], &p[4 * a])) > 1e-10 * ecm * ecm)"),
    ("heavy-jet mass as the lighter hemisphere", "double rho = (mp > mm ? mp : mm) / s;",
     "double rho = (mp < mm ? mp : mm) / s;"),
    ("validation always DONE", "  double tot[4] = {0, 0, 0, 0};\n  for (int a = 0; a < 4 * n; ++a)",
     "  return OR_DONE;\n  double tot[4] = {0, 0, 0, 0};\n  for (int a = 0; a < 4 * n; ++a)"),
    ("validation tolerance not scaled by sqrt(s)", "double tol = 1e-10 * ecm;", "double tol = 1e-10;"),
    ("validation tolerance scaled by s", "double tol = 1e-10 * ecm;", "double tol = 1e-10 * ecm * ecm;"),
    ("validation: massless partons' shells unchecked",
     "if (fabs(mdot(&p[4 * a], &p[4 * a]) - m * m) > 1e-10 * ecm * ecm)",
     "if (m > 0.0 && fabs(mdot(&p[4 * a], &p[4 * a]) - m * m) > 1e-10 * ecm * ecm)"),
    ("validation: a non-finite component reported as non-conservation", "if (!isfinite(p[a])) return OR_NONFINITE;",
     "if (!isfinite(p[a])) return OR_CONSERVATION;"),
    ("q->qg soft term without y", "if (K < 10) return CF * (2.0 / (1.0 - z * (1.0 - y)) - (1.0 + z));",
     "if (K < 10) return CF * (2.0 / (1.0 - z) - (1.0 + z));"),
    ("g->gg soft term without y", "if (K == 10) return 0.5 * CA * (2.0 / (1.0 - z * (1.0 - y))",
     "if (K == 10) return 0.5 * CA * (2.0 / (1.0 - z)"),
    ("massive map: kT^2 not clamped at the edge", "double kt = sqrt(k2 > 0.0 ? k2 : 0.0)", "double kt = sqrt(k2)"),
    ("ISR: PDF ratio dropped", "double dens = p / z * or_pdf_q(x / z) / or_pdf_q(x);", "double dens = p / z;"),
    ("ISR: 1/z of the backward density dropped", "double dens = p / z * or_pdf_q(x / z) / or_pdf_q(x);",
     "double dens = p * or_pdf_q(x / z) / or_pdf_q(x);"),
    ("ISR: overestimate without x^(-1/2)", "double over = 2.0 * CF / sqrt(x) / (1.0 - z);",
     "double over = 2.0 * CF / (1.0 - z);"),
    ("ISR: the spectator's fraction in the PDF ratio", "double r = or_isr_ratio(t, z, x[wl], st);",
     "double r = or_isr_ratio(t, z, x[1 - wl], st);"),
    ("ISR: emitter's fraction not rescaled", "    x[wl] /= z;\n", "    x[wl] *= 1.0;\n"),
    ("ISR: the larger root of v", "double v = 0.5 * ((1.0 - z) - sqrt(", "double v = 0.5 * ((1.0 - z) + sqrt("),
    ("ISR: final state not boosted", "for (int m = 0; m < 4; ++m) x[m] = y[m];", "(void)y;"),
    ("ISR: gluon density normalisation", "return x > 0.0 && x < 1.0 ? 3.0 / x * pow(1.0 - x, 5.0) : 0.0;",
     "return x > 0.0 && x < 1.0 ? 2.0 / x * pow(1.0 - x, 5.0) : 0.0;"),
    ("ISR: tau taken as Q / sqrt(S)", "double tau = q * q / (sqrt_s_had * sqrt_s_had);", "double tau = q / sqrt_s_had;"),
]


def test_every_mutation_site_is_unique():
    src = open(SRC).read()
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once"
        assert old != new


def _build(src_text, out):
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "vsh_oracle.c")
        open(c, "w").write(src_text)
        subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                        "-I", os.path.dirname(SRC), "-o", out, c, "-lm"], check=True, capture_output=True)


def _run_pins(lib):
    env = dict(os.environ, VSH_ORACLE_LIB=lib)
    p = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    lines = [ln for ln in p.stdout.splitlines() if ln.startswith("FAILED") or ln.startswith("ERROR")]
    return p.returncode, lines[0] if lines else p.stdout.strip().splitlines()[-1]


@pytest.mark.slow
def test_pins_kill_every_mutant(tmp_path):
    src = open(SRC).read()

    def one(k):
        name, old, new = MUTANTS[k]
        lib = str(tmp_path / f"mutant_{k}.so")
        _build(src.replace(old, new), lib)
        return name, _run_pins(lib)

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(one, range(len(MUTANTS))))
    survivors = [name for name, (rc, _) in results if rc == 0]
    for name, (rc, line) in results:
        print(f"{'killed ' if rc else 'SURVIVED'} {name}: {line}")
    assert not survivors, f"mutants not caught by any pin: {survivors}"
