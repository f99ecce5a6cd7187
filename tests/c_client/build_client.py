"""Build the plain-C client of the library's ABI (sph_abi_client.c) with gcc
in strict C99: the header must compile as C, and the client links against
libsph.so and the HIP runtime only.  Usage: python tests/c_client/build_client.py [OUT]."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BIN = os.path.join(HERE, "sph_abi_client")


def build(out: str = BIN) -> str:
    pkg = os.path.join(ROOT, "paper_2606_23891_amd")
    rel = os.path.relpath(pkg, os.path.dirname(os.path.abspath(out)))
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-pedantic", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "sph_abi_client.c"), "-o", out, "-L", pkg, "-lsph",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,$ORIGIN/{rel}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for the ABI client:\n" + r.stderr)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else BIN))
