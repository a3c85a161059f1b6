import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NATIVE = os.path.join(ROOT, "tests", "native")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU statistics")


@pytest.fixture(scope="session")
def native_bin(tmp_path_factory):
    """Compiles a helper under tests/native/ on first use; returns its path."""
    out_dir = tmp_path_factory.mktemp("native")
    built = {}

    def get(name: str) -> str:
        if name in built:
            return built[name]
        src = os.path.join(NATIVE, name)
        exe = str(out_dir / os.path.splitext(name)[0])
        if name.endswith(".cpp"):
            import torch

            inc = os.path.join(os.path.dirname(torch.__file__), "include")
            cmd = ["g++", "-std=c++17", "-O2", "-I", inc, "-o", exe, src]
        else:
            cmd = ["gcc", "-std=c11", "-O3", "-o", exe, src, "-lm"]
        subprocess.run(cmd, check=True)
        built[name] = exe
        return exe

    return get


def have_gpu() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle._load()
    return oracle
