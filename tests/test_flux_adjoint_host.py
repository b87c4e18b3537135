"""Host self-check of the reverse flux products used by the GPU vector-Jacobian product:
the header's transposed-Jacobian products against central differences of its forward fluxes
(Euler, KEP, central, Roe dissipation, LLF/Roe Riemann solvers, viscous flux, variable maps)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "flux_selftest.cpp")


def test_flux_adjoints_match_finite_differences(tmp_path):
    exe = str(tmp_path / "flux_selftest")
    subprocess.run(["g++", "-O2", "-std=c++17", SRC, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
