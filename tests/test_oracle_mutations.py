"""Mutation check of the oracle's encoder pins (Sec. 5.1): one mistake at a time is planted in a
copy of the oracle's C source, the copy is built, and tests/test_oracle_encoder.py must fail on
it.  The unmutated copy must pass, so a failure comes from the planted mistake.  CPU only; the
repository's own oracle is never changed."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in the oracle source, its replacement); every text occurs exactly once
MUTATIONS = [
    ("ReLU on the encoder's output layer",
     "            act[k][o] = (k < KE) ? (s > 0.0 ? s : 0.0) : s;",
     "            act[k][o] = (s > 0.0 ? s : 0.0);"),
    ("no ReLU on the encoder's hidden layers",
     "            act[k][o] = (k < KE) ? (s > 0.0 ? s : 0.0) : s;",
     "            act[k][o] = s;"),
    ("transposed encoder weights",
     "            for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * act[k - 1][j];\n            act[k][o] = (k < KE)",
     "            for (int j = 0; j < fi; ++j) s += W[(long)j * fo + o] * act[k - 1][j];\n            act[k][o] = (k < KE)"),
    ("encoder bias dropped",
     "            double s = b[o];\n            for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * act[k - 1][j];",
     "            double s = 0.0 * b[o];\n            for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * act[k - 1][j];"),
    ("code gradient with the wrong sign",
     "            for (int c = 0; c < C; ++c) dz[(long)C * i + c] = d[c];",
     "            for (int c = 0; c < C; ++c) dz[(long)C * i + c] = -d[c];"),
    ("non-finite code not skipped",
     "            for (int c = 0; c < C; ++c) dz[(long)C * i + c] = 0.0;\n            if (!finite) continue;",
     "            for (int c = 0; c < C; ++c) dz[(long)C * i + c] = 0.0;\n            if (!finite && finite) continue;"),
    ("encoder backward without the ReLU derivative",
     "                    dprev[j] = (a_in[j] > 0.0) ? s : 0.0;",
     "                    dprev[j] = s;"),
    ("encoder bias gradient doubled",
     "                    gb[r] += d[r];\n                    for (int j = 0; j < fi; ++j) gW[(long)r * fi + j] += d[r] * a_in[j];\n"
     "                }\n                if (k == 1) break;",
     "                    gb[r] += 2.0 * d[r];\n                    for (int j = 0; j < fi; ++j) gW[(long)r * fi + j] += d[r] * a_in[j];\n"
     "                }\n                if (k == 1) break;"),
    ("encoder backward through transposed weights",
     "                    for (int r = 0; r < fo; ++r) s += W[(long)r * fi + j] * d[r];\n                    dprev[j] = (a_in[j] > 0.0)",
     "                    for (int r = 0; r < fo; ++r) s += W[(long)j * fo + r] * d[r];\n                    dprev[j] = (a_in[j] > 0.0)"),
]


def _run_pins(tree, source):
    """Copy of the repository's tests and oracle (with `source` as its C file) under `tree`, the
    package linked; returns the exit status of the encoder pins run there."""
    os.makedirs(os.path.join(tree, "oracle"))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(tree, "tests"))
    os.symlink(os.path.join(ROOT, "paper_2305_02678_amd"), os.path.join(tree, "paper_2305_02678_amd"))
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), os.path.join(tree, "oracle", "__init__.py"))
    with open(os.path.join(tree, "oracle", "nam_oracle.c"), "w") as f:
        f.write(source)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(tree, "tests", "test_oracle_encoder.py")],
                       capture_output=True, text=True, cwd=tree, timeout=300)
    return r.returncode


def _source():
    with open(os.path.join(ROOT, "oracle", "nam_oracle.c")) as f:
        return f.read()


def test_unmutated_copy_passes(tmp_path):
    assert _run_pins(str(tmp_path / "tree"), _source()) == 0


@pytest.mark.parametrize("name,text,replacement", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, text, replacement):
    src = _source()
    assert src.count(text) == 1, name
    assert _run_pins(str(tmp_path / "tree"), src.replace(text, replacement)) != 0, name
