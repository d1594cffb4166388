"""The library driven from C through its ABI alone (tests/c_abi/step_from_c.c,
built with gcc against include/pic.h, libpic.so and the HIP runtime): the
host-only configuration checks on the CPU, and on the GPU a short run of
free-streaming particles whose total current and final positions have
closed forms.  No Python marshalling is involved on the C side."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2204_12837_amd")
ROCM = "/opt/rocm"


def _build(tmp_path):
    if shutil.which("gcc") is None or not os.path.exists(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs gcc and the HIP headers")
    if not os.path.exists(os.path.join(PKG, "libpic.so")):
        pytest.skip("libpic.so is not built")
    exe = str(tmp_path / "step_from_c")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "c_abi", "step_from_c.c"), "-o", exe,
                    "-L", PKG, "-lpic", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
                    f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"], check=True)
    return exe


def test_c_program_host_checks(tmp_path):
    exe = _build(tmp_path)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok"), out.stdout


@pytest.mark.gpu
def test_c_program_steps_on_the_gpu(tmp_path):
    exe = _build(tmp_path)
    print("case c-abi program", flush=True)
    out = subprocess.run([exe, "gpu"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok"), out.stdout
