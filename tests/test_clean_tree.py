"""A tree without any built library must still build: the build module and the
package import without libsrmdp.so, and the binding fails loudly (ImportError)
until the library exists.  Runs on the CPU, compiles nothing."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tracked_files():
    try:
        out = subprocess.run(["git", "-C", ROOT, "ls-files"], capture_output=True, text=True, check=True)
        files = [f for f in out.stdout.splitlines() if f]
        if files:
            return files
    except (OSError, subprocess.CalledProcessError):
        pass
    skip_dirs = {".git", "__pycache__", "gpurun_out", "_work", ".pytest_cache"}
    files = []
    for base, dirs, names in os.walk(ROOT):
        dirs[:] = [d for d in dirs if d not in skip_dirs]
        for n in names:
            if not n.endswith((".so", ".srchash", ".pyc")):
                files.append(os.path.relpath(os.path.join(base, n), ROOT))
    return files


@pytest.fixture(scope="module")
def clean_copy(tmp_path_factory):
    dst = tmp_path_factory.mktemp("clean_tree")
    for rel in _tracked_files():
        src = os.path.join(ROOT, rel)
        if not os.path.isfile(src):
            continue
        os.makedirs(os.path.join(dst, os.path.dirname(rel)), exist_ok=True)
        shutil.copy2(src, os.path.join(dst, rel))
    assert not os.path.exists(os.path.join(dst, "paper_2407_21085_amd", "libsrmdp.so"))
    return str(dst)


def _run(cwd, code):
    env = dict(os.environ, PYTHONPATH=cwd, PYTHONDONTWRITEBYTECODE="1")
    return subprocess.run([sys.executable, "-c", code], cwd=cwd, env=env, capture_output=True, text=True)


def test_build_module_imports_without_the_library(clean_copy):
    res = _run(clean_copy, (
        "import paper_2407_21085_amd.build as B, os\n"
        "assert B.LIB_PATH.startswith(os.getcwd()), B.LIB_PATH\n"
        "assert B.is_stale()\n"
        "assert len(B.source_hash()) == 64\n"
        "import __graft_entry__\n"
        "print('ok')\n"))
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok")


def test_binding_fails_loudly_without_the_library(clean_copy):
    res = _run(clean_copy, (
        "import paper_2407_21085_amd as S\n"
        "try:\n"
        "    S.solve\n"
        "except ImportError as e:\n"
        "    print('ImportError:', e)\n"
        "else:\n"
        "    raise SystemExit('the binding loaded without a library')\n"))
    assert res.returncode == 0, res.stdout + res.stderr
    assert "libsrmdp.so is missing" in res.stdout


def test_source_hash_is_independent_of_the_tree_location(clean_copy):
    here = _run(ROOT, "import paper_2407_21085_amd.build as B; print(B.source_hash())")
    there = _run(clean_copy, "import paper_2407_21085_amd.build as B; print(B.source_hash())")
    assert here.returncode == 0 and there.returncode == 0, here.stderr + there.stderr
    if subprocess.run(["git", "-C", ROOT, "diff", "--quiet", "--", "paper_2407_21085_amd/csrc",
                       "include", "paper_2407_21085_amd/build.py"]).returncode == 0:
        assert here.stdout.strip() == there.stdout.strip()
