"""The process holds exactly one HIP runtime after the binding is imported
(torch's), whatever was imported first."""
import subprocess
import sys
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_single_hip_runtime_when_binding_imported_first():
    code = ("import paper_2204_08147_amd, torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
            "print(len(libs)); print(libs)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.splitlines()[0] == "1", out.stdout
