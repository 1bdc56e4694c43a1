"""The oracle's pins reject plausible mistakes: each entry below plants one mistake in a copy
of oracle.cpp (on the CPU), builds it, and runs the pin suite against it; every mutant must
fail at least one pin."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "rotation block sign": ("R[d][b] = s;   // sigma_b -> c sigma_b + s sigma_d", "R[d][b] = -s;"),
    "rotation block transposed": ("R[b][d] = -s;  // sigma_d -> c sigma_d - s sigma_b", "R[b][d] = s;"),
    "CX without sign": ("bool flip = (xc & zt & (xt ^ zc ^ 1u)) != 0;", "bool flip = false;"),
    "CX control/target swapped": ("xt ^= xc;\n  zc ^= zt;", "zt ^= zc;\n  xc ^= xt;"),
    "no merge of equal strings": ("while (j < images.size() && images[j].x == acc.x && images[j].z == acc.z) {",
                                  "while (false) {"),
    "H keeps Y": ("case G_H: R[3][1] = 1; R[2][2] = -1; R[1][3] = 1;", "case G_H: R[3][1] = 1; R[2][2] = 1; R[1][3] = 1;"),
    "S turns the other way": ("case G_S: R[2][1] = 1; R[1][2] = -1; R[3][3] = 1;",
                              "case G_S: R[2][1] = -1; R[1][2] = 1; R[3][3] = 1;"),
    "SX sign": ("case G_SX: R[1][1] = 1; R[3][2] = 1; R[2][3] = -1;", "case G_SX: R[1][1] = 1; R[3][2] = -1; R[2][3] = 1;"),
    "exact zeros kept": ("if (acc.w != 0.0) out.push_back(acc);", "out.push_back(acc);"),
    "prune keeps |w| == eps": ("if (std::fabs(gen[i].w) > eps) gen[k++] = gen[i];",
                               "if (std::fabs(gen[i].w) >= eps) gen[k++] = gen[i];"),
    "Y and Z codes swapped": ("if (xb && zb) return 2;\n  return 3;", "if (xb && zb) return 3;\n  return 2;"),
    "generators start as X": ("g[0].z = 1ull << j;  // Z on qubit j", "g[0].x = 1ull << j; g[0].z = 0;"),
    "two-qubit rotation image sign": ("u.w = t.w * s * (k == 0 ? 1.0 : -1.0);", "u.w = t.w * s * (k == 0 ? -1.0 : 1.0);"),
    "two-qubit rotation commutation test": ("const int sym = ((xa & pz) ^ (za & px)) ^ ((xb & pz) ^ (zb & px));",
                                            "const int sym = ((xa & pz) ^ (za & px)) | ((xb & pz) ^ (zb & px));"),
    "ISWAP as XX only": ("      apply_pp_rotation(gen, a, b, 1, 1, 0.0, -1.0, scratch);  // exp(i pi/4 YY)\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_mutant(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "oracle.cpp")).read()
    old, new = MUTATIONS[name]
    assert old in src, f"mutation site not found: {name}"
    cpp = tmp_path / "mutant.cpp"
    so = tmp_path / "mutant.so"
    cpp.write_text(src.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", str(so), str(cpp)], check=True)
    env = dict(os.environ, QIMAX_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-x"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught the mutant '{name}'"
