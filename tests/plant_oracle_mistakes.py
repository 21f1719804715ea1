"""Planted-mistake check of the oracle's pins (a script, not collected by pytest: it takes about
20 minutes on 8 cores).

Each entry below changes one coefficient, sign or index of the oracle's arithmetic -- the BSSN
right-hand side (section "Basic equations"), the radiation fluid's sources, fluxes and
characteristic speeds, the Kurganov-Tadmor numerical flux and reconstruction, the scalar field's
wave operator, the constraints, the Kreiss-Oliger and upwind stencils. For each, the script copies
`oracle/` and `tests/` into a temporary folder, applies the change to the copy's
`cosmos_oracle.hpp`, builds it and runs the CPU pin tests (`tests/test_oracle_*.py`, slow ones
included) against it. A mutation is caught when a pin test fails. Nothing outside the temporary
copy is touched.

Usage: python tests/plant_oracle_mistakes.py [name ...]   (no names: all)
"""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, the oracle's text, the planted mistake)
MUTATIONS = [
    ("chi_rhs", "out[CHI] = T(2.0 / 3.0) * chi * (alpha * K - divb);",
     "out[CHI] = T(1.0 / 3.0) * chi * (alpha * K - divb);"),
    ("gt_At", "- T(2.0) * alpha * in.At[s];", "- T(1.0) * alpha * in.At[s];"),
    ("K_KK", "alpha * (AA + K * K / T(3.0))", "alpha * (AA + K * K / T(2.0))"),
    ("K_matter", "pi4 * alpha * EpS", "pi8 * alpha * EpS"),
    ("At_Sij", "- pi8 * (sc ? M.Sij[s] + X.Sij[s] : M.Sij[s])", "- pi4 * (sc ? M.Sij[s] + X.Sij[s] : M.Sij[s])"),
    ("At_divb", "acc = acc - T(2.0 / 3.0) * in.At[s] * divb;", "acc = acc - T(1.0 / 3.0) * in.At[s] * divb;"),
    ("At_AA", "out[AT + s] = acc + alpha * (K * in.At[s] - T(2.0) * AAij);",
     "out[AT + s] = acc + alpha * (K * in.At[s] - T(1.0) * AAij);"),
    ("Gam_divb", "acc = acc + T(2.0 / 3.0) * G.Gd[i] * divb;", "acc = acc + T(1.0 / 3.0) * G.Gd[i] * divb;"),
    ("Gam_d2beta", "in.d2beta[k][SYM[j][k]] / T(3.0);", "in.d2beta[k][SYM[j][k]] / T(2.0);"),
    ("Gam_dchi", "inner = inner - T(1.5) * Aup[SYM[i][j]] * in.dchi[j] / chi;",
     "inner = inner - T(1.0) * Aup[SYM[i][j]] * in.dchi[j] / chi;"),
    ("Gam_dK", "inner = inner - T(2.0 / 3.0) * gi[SYM[i][j]] * in.dK[j];",
     "inner = inner - T(4.0 / 3.0) * gi[SYM[i][j]] * in.dK[j];"),
    ("Gam_S", "out[GAM + i] = acc - pi16 * alpha * gS;", "out[GAM + i] = acc - pi8 * alpha * gS;"),
    ("Gam_Gd", "for (int k = 0; k < 3; ++k) acc = acc - G.Gd[k] * in.dbeta[i][k];",
     "for (int k = 0; k < 3; ++k) acc = acc + G.Gd[k] * in.dbeta[i][k];"),
    ("Gam_Adalpha", "for (int j = 0; j < 3; ++j) acc = acc - T(2.0) * Aup[SYM[i][j]] * in.dalpha[j];",
     "for (int j = 0; j < 3; ++j) acc = acc - T(1.0) * Aup[SYM[i][j]] * in.dalpha[j];"),
    ("lapse", "out[ALP] = T(-2.0) * alpha * (K - T(K_background(p, t)));",
     "out[ALP] = T(-1.0) * alpha * (K - T(K_background(p, t)));"),
    ("shift", "T(0.75) * in.Gam[i] - T(p.eta) * in.beta[i]", "T(0.5) * in.Gam[i] - T(p.eta) * in.beta[i]"),
    ("Et_Sda", "out[ET] = im32 * (alpha * KS - Sda);", "out[ET] = im32 * (alpha * KS + Sda);"),
    ("St_Edalpha", "T acc = -M.E * in.dalpha[i];", "T acc = M.E * in.dalpha[i];"),
    ("St_sg", "out[ST + i] = im32 * (acc + alpha / T(2.0) * sg);", "out[ST + i] = im32 * (acc + alpha / T(4.0) * sg);"),
    ("St_Sdbeta", "for (int k = 0; k < 3; ++k) acc = acc + M.S[k] * in.dbeta[k][i];",
     "for (int k = 0; k < 3; ++k) acc = acc + M.S[i] * in.dbeta[k][i];"),
    ("Pi_dad", "sout[PIF] = alpha * K * sc->Pi + alpha * chi * lap + chi * dad;",
     "sout[PIF] = alpha * K * sc->Pi + alpha * chi * lap + T(2.0) * chi * dad;"),
    ("Pi_gk", "for (int l = 0; l < 3; ++l) gk = gk + gi[SYM[k][l]] * in.dchi[l] / (T(2.0) * chi);",
     "for (int l = 0; l < 3; ++l) gk = gk + gi[SYM[k][l]] * in.dchi[l] / (T(4.0) * chi);"),
    ("flux_beta", "out[4 * j] = im32 * (alpha * M.Sup[j] - beta[j] * M.E);",
     "out[4 * j] = im32 * (alpha * M.Sup[j] + beta[j] * M.E);"),
    ("flux_P", "T pd = (i == j) ? M.P : T(0.0);", "T pd = (i == j) ? T(2.0) * M.P : T(0.0);"),
    ("H_KK", "H = G.R + T(2.0 / 3.0) * in.K * in.K - AA - T(16.0 * PI) * Mt.E;",
     "H = G.R + T(1.0 / 3.0) * in.K * in.K - AA - T(16.0 * PI) * Mt.E;"),
    ("M_S", "acc = acc - T(2.0 / 3.0) * in.dK[i] - T(8.0 * PI) * Mt.S[i];",
     "acc = acc - T(2.0 / 3.0) * in.dK[i] - T(4.0 * PI) * Mt.S[i];"),
    ("M_dchi", "for (int j = 0; j < 3; ++j) acc = acc - T(1.5) * Amix[j][i] * in.dchi[j] / in.chi;",
     "for (int j = 0; j < 3; ++j) acc = acc - T(1.0) * Amix[j][i] * in.dchi[j] / in.chi;"),
    ("KO_coef", "return T(eps / 64.0) * s;", "return T(eps / 32.0) * s;"),
    ("upwind", "static constexpr double CUP[5] = {-3.0, -10.0, 18.0, -6.0, 1.0};",
     "static constexpr double CUP[5] = {-1.0, -10.0, 18.0, -6.0, -1.0};"),
    ("KT_slope", "uL[f] = q0 + T(0.5) * s0;", "uL[f] = q0 + T(0.25) * s0;"),
    ("KT_c", "out[q] = T(0.5) * (FL[4 * a + q] + FR[4 * a + q]) - T(0.5) * c * (uR[ET + q] - uL[ET + q]);",
     "out[q] = T(0.5) * (FL[4 * a + q] + FR[4 * a + q]) - T(0.25) * c * (uR[ET + q] - uL[ET + q]);"),
    ("speed_root", "lp = f * (va * (T(1.0) - cs2) + cs * root) - u[BET + a];",
     "lp = f * (va * (T(1.0) - cs2) + root) - u[BET + a];"),
    ("Strace", "M.Strace = M.S2 * M.invX + T(3.0) * M.P;", "M.Strace = M.S2 * M.invX + T(2.0) * M.P;"),
]
# Not listed: the pressure part of S_ij (P gamma_ij) is pure trace, which the trace-free projection
# of the A~ source removes, so changing it changes no result (only the stored operation count).

PIN_TESTS = ["tests/test_oracle_physics.py", "tests/test_oracle_algebra.py", "tests/test_oracle_stencils.py",
             "tests/test_oracle_gauge.py", "tests/test_oracle_kt.py", "tests/test_oracle_scalar.py",
             "tests/test_oracle_ad.py", "tests/test_oracle_linear_mode.py"]


def run(name: str, old: str, new: str, scratch: str) -> bool:
    d = os.path.join(scratch, name)
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(d, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(d, "tests"), ignore=shutil.ignore_patterns("__pycache__"))
    src = os.path.join(d, "oracle", "cosmos_oracle.hpp")
    text = open(src).read()
    if text.count(old) != 1:
        raise SystemExit(f"{name}: the oracle text to change occurs {text.count(old)} times")
    open(src, "w").write(text.replace(old, new))
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build()"], cwd=d, check=True, capture_output=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
                       + PIN_TESTS, cwd=d, capture_output=True, text=True)
    failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    print(f"{name:12s} {'caught by ' + failed[0] if r.returncode else 'MISSED'}", flush=True)
    shutil.rmtree(d)
    return r.returncode != 0


def main(names):
    chosen = [m for m in MUTATIONS if not names or m[0] in names]
    with tempfile.TemporaryDirectory() as scratch:
        missed = [m[0] for m in chosen if not run(*m, scratch)]
    print(f"{len(chosen) - len(missed)} of {len(chosen)} caught" + (f"; missed: {missed}" if missed else ""))
    return 1 if missed else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
