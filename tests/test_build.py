"""The build entry point works from a checkout with no built library (the
package loads libsrf.so at import, so the build script must not need the
package): a copy of the sources without any .so is built and imported in a
fresh process.  Host only (hipcc cross-compiles for gfx950)."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_from_a_clean_copy(tmp_path):
    ignore = shutil.ignore_patterns("*.so", "*.so.tmp", "_build", "__pycache__", "*.o")
    for d in ("paper_1211_4406_amd", "include", "oracle"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d, ignore=ignore)
    shutil.copy(os.path.join(ROOT, "__graft_entry__.py"), tmp_path / "__graft_entry__.py")
    assert not list(tmp_path.rglob("*.so"))
    code = ("import __graft_entry__ as g; g.build(); import paper_1211_4406_amd as s; "
            "print(s.lib_path())")
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == str(tmp_path / "paper_1211_4406_amd" / "libsrf.so")
    assert (tmp_path / "oracle" / "liboracle.so").exists()
