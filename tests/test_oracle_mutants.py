"""The pins of tests/test_oracle_pins.py must catch plausible mistakes.

Each case plants one mistake in a scratch copy of the oracle's C source (a
twist factor conjugated or moved, a leaf mis-oriented, an RK3 coefficient, a
normalisation, a sign, a neighbour index, the schedule; for the Monte Carlo a
subgroup vector, the heat-bath coupling, an acceptance test, the direction
draw, the checkerboard, the SU(2) embedding; for SU(N) the twist phase, the
trace part, the normalisations, a staple factor, the exponential, RK3, the
twist modulus), rebuilds it, and requires the pin suite of that part
(tests/test_oracle_pins.py, tests/test_oracle_mc.py, tests/test_oracle_sun.py)
to fail.  CPU only; the real oracle is untouched.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("lower staple factor conjugated",
     "om = m_add(om, m_scale(zfac(L, imn, mu, nu), lo));",
     "om = m_add(om, m_scale(conj(zfac(L, imn, mu, nu)), lo));"),
    ("upper factor not conjugated",
     "om = m_add(om, m_scale(conj(zfac(L, i, mu, nu)), up));",
     "om = m_add(om, m_scale(zfac(L, i, mu, nu), up));"),
    ("RK3 17/36 -> 17/9", "m_scale(-17.0 / 36.0, Z0[l])", "m_scale(-17.0 / 9.0, Z0[l])"),
    ("RK3 3/4 -> 1/4", "m_scale(0.75, Z2[l])", "m_scale(0.25, Z2[l])"),
    ("clover 1/8 -> 1/4", "(-I / 8.0)", "(-I / 4.0)"),
    ("leaf 3 twist base n-nu",
     "C = m_add(C, m_scale(conj(zfac(L, i_m, mu, nu)), plaq_s(L, links, i, pn, mm)));",
     "C = m_add(C, m_scale(conj(zfac(L, i_n, mu, nu)), plaq_s(L, links, i, pn, mm)));"),
    ("leaf 2 orientation flipped", "plaq_s(L, links, i, mn, pm)", "plaq_s(L, links, i, pm, mn)"),
    ("no trace subtraction in P_ah", "for (int i = 0; i < 3; i++) r.a[i][i] -= t;", "(void)t;"),
    ("force sign",
     "F[i * 4 + mu] = m_scale(-1.0, m_proj_ah(omega(L, links, i, mu)));",
     "F[i * 4 + mu] = m_proj_ah(omega(L, links, i, mu));"),
    ("exponential truncated", "for (int k = 1; k <= 16; k++) {", "for (int k = 1; k <= 2; k++) {"),
    ("twist site shifted",
     "if (n[mu] != L->base[mu] || n[nu] != L->base[nu]) return 1.0;",
     "if (n[mu] != L->base[mu] || n[nu] != (L->base[nu] + 1) % L->d[nu]) return 1.0;"),
    ("Levi-Civita sign", "q += 0.5 * eps * creal", "q -= 0.5 * eps * creal"),
    ("E factor 1/2 dropped", "e += 0.5 * creal(m_tr(m_mul(G[m][n], G[m][n])));",
     "e += creal(m_tr(m_mul(G[m][n], G[m][n])));"),
    ("plaquette normalisation", "out[1] = p / (18.0 * V);", "out[1] = p / (9.0 * V);"),
    ("lower staple neighbour", "long ipm_mn = step(L, ipm, nu, -1);", "long ipm_mn = step(L, i, nu, -1);"),
    ("no short final step", "int has_short = (t_end - t_last) > 1e-12;", "int has_short = 0;"),
    # another three-stage scheme of third order on the group (nodes 1/3, 3/4,
    # weights 1/6, 3/10, 8/15): the order test and the single-mode decay pass
    # it, only the torus reduction to Luscher's tableau tells it apart
    ("RK3 another third-order scheme",
     ["W[l] = m_mul(m_exp(m_scale(0.25, Z0[l])), W[l]);",
      "mat A = m_add(m_scale(8.0 / 9.0, Z1[l]), m_scale(-17.0 / 36.0, Z0[l]));",
      "m_scale(0.75, Z2[l]), m_scale(-8.0 / 9.0, Z1[l])),\n                      "
      "m_scale(17.0 / 36.0, Z0[l])"],
     ["W[l] = m_mul(m_exp(m_scale(1.0 / 3.0, Z0[l])), W[l]);",
      "mat A = m_add(m_scale(15.0 / 16.0, Z1[l]), m_scale(-25.0 / 48.0, Z0[l]));",
      "m_scale(8.0 / 15.0, Z2[l]), m_scale(-51.0 / 80.0, Z1[l])),\n                      "
      "m_scale(17.0 / 48.0, Z0[l])"]),
]

# Monte Carlo mistakes, caught by tests/test_oracle_mc.py
MC_MUTANTS = [
    ("subgroup vector component sign",
     "c[2] = creal(W.a[b][a]) - creal(W.a[a][b]);", "c[2] = creal(W.a[a][b]) - creal(W.a[b][a]);"),
    ("heat-bath alpha halved", "su2_draw(beta * k / 3.0,", "su2_draw(beta * k / 6.0,"),
    ("Kennedy-Pendleton acceptance", "ok = u4_ * u4_ <= 1.0 - X;", "ok = u4_ <= 1.0 - X;"),
    ("Creutz acceptance", "ok = u2 * u2 <= 1.0 - y0 * y0;\n        } else {",
     "ok = u2 <= 1.0 - y0 * y0;\n        } else {"),
    ("direction on a hemisphere", "double ct = 2.0 * u01(r.v[0]) - 1.0,", "double ct = u01(r.v[0]),"),
    ("no checkerboard", "if (((n[0] + n[1] + n[2] + n[3]) & 1) != par) continue;",
     "if (par) continue;"),
    ("SU(2) embedding sign", "m[0][1] = a[2] + I * a[1];", "m[0][1] = -a[2] + I * a[1];"),
    ("staple not updated between subgroups", "rows_mul(&W, a, b, A);", "(void)W;"),
]

# SU(N) mistakes (oracle/sun_oracle.c), caught by tests/test_oracle_sun.py
SUN_MUTANTS = [
    ("SU(N) twist phase with N = 3", "cexp(I * (2.0 * PI * L->tw[mu][nu] / L->n))",
     "cexp(I * (2.0 * PI * L->tw[mu][nu] / 3.0))"),
    ("SU(N) trace part 1/3", "cplx t = z_tr(n, &r) / (double)n;", "cplx t = z_tr(n, &r) / 3.0;"),
    ("SU(N) plaquette normalisation", "out[1] = psum(d + 2, V, 4) / (6.0 * L->n * V);",
     "out[1] = psum(d + 2, V, 4) / (18.0 * V);"),
    ("SU(N) action constant", "s += n - re;", "s += 3 - re;"),
    ("SU(N) lower staple factor conjugated", "z_axpy(n, zf(L, imn, mu, nu), &lo, &om);",
     "z_axpy(n, conj(zf(L, imn, mu, nu)), &lo, &om);"),
    ("SU(N) exponential truncated", "for (int k = 1; k <= 20; k++) {", "for (int k = 1; k <= 3; k++) {"),
    ("SU(N) RK3 17/36 -> 17/9", "{-17.0 / 36.0, 8.0 / 9.0, 0}", "{-17.0 / 9.0, 8.0 / 9.0, 0}"),
    ("SU(N) RK3 another third-order scheme",
     "{{0.25, 0, 0}, {-17.0 / 36.0, 8.0 / 9.0, 0}, {17.0 / 36.0, -8.0 / 9.0, 0.75}}",
     "{{1.0 / 3.0, 0, 0}, {-25.0 / 48.0, 15.0 / 16.0, 0}, {17.0 / 48.0, -51.0 / 80.0, 8.0 / 15.0}}"),
    ("SU(N) twist taken mod 3", "int t = twist6 ? ((twist6[k] % nc) + nc) % nc : 0;",
     "int t = twist6 ? ((twist6[k] % 3) + 3) % 3 : 0;"),
]


def _run_mutant(tmp_path, name, old, new, pins, source="tgf_oracle.c"):
    for sub in ("oracle", "tests", "paper_2107_03747_amd"):
        shutil.copytree(os.path.join(ROOT, sub), tmp_path / sub,
                        ignore=shutil.ignore_patterns("*.so", "*.so.tmp", "__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), tmp_path)
    src = tmp_path / "oracle" / source
    text = src.read_text()
    olds, news = ([old], [new]) if isinstance(old, str) else (old, new)
    for o, n in zip(olds, news):
        assert text.count(o) >= 1, f"mutation site for '{name}' not found: {o}"
        text = text.replace(o, n, 1)
    src.write_text(text)
    r = subprocess.run([sys.executable, "-m", "pytest", pins, "-q", "-x",
                        "-p", "no:cacheprovider"], cwd=tmp_path, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode != 0, f"planted mistake '{name}' was not caught:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    _run_mutant(tmp_path, name, old, new, "tests/test_oracle_pins.py")


@pytest.mark.parametrize("name,old,new", MC_MUTANTS, ids=[m[0] for m in MC_MUTANTS])
def test_mc_pins_catch_planted_mistake(tmp_path, name, old, new):
    _run_mutant(tmp_path, name, old, new, "tests/test_oracle_mc.py")


@pytest.mark.parametrize("name,old,new", SUN_MUTANTS, ids=[m[0] for m in SUN_MUTANTS])
def test_sun_pins_catch_planted_mistake(tmp_path, name, old, new):
    _run_mutant(tmp_path, name, old, new, "tests/test_oracle_sun.py", source="sun_oracle.c")
