"""The product path (the package under paper_2312_00005_amd) never imports the
oracle: importing every module of the package in a fresh interpreter leaves no
oracle module loaded, and no package source names it in an import."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2312_00005_amd")


def test_package_modules_do_not_load_the_oracle():
    code = ("import sys\n"
            "import paper_2312_00005_amd.bemfmm, paper_2312_00005_amd.sweep, paper_2312_00005_amd.adjoint, "
            "paper_2312_00005_amd.curves\n"
            "bad = sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.'))\n"
            "print(bad)\n"
            "sys.exit(1 if bad else 0)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_package_sources_have_no_oracle_import():
    pat = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b)", re.M)
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith(".py"):
                with open(os.path.join(dirpath, f)) as fh:
                    assert not pat.search(fh.read()), os.path.join(dirpath, f)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libbemfmm.so cannot be imported: there is
    no fallback path."""
    import shutil
    dst = tmp_path / "paper_2312_00005_amd"
    dst.mkdir()
    for f in os.listdir(PKG):
        if f.endswith(".py"):
            shutil.copy(os.path.join(PKG, f), dst / f)
    code = ("import sys\n"
            f"sys.path.insert(0, {str(tmp_path)!r})\n"
            "try:\n"
            "    import paper_2312_00005_amd.bemfmm as b\n"
            "except ImportError as e:\n"
            "    print('ImportError:', e)\n"
            "    sys.exit(0)\n"
            "print('imported', b.__file__)\n"
            "sys.exit(1)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "libbemfmm.so is missing" in r.stdout
