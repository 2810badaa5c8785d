"""Builds the oracle's C library (test infrastructure, see oracle/__init__.py)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "sph_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")


def library_path() -> str:
    return os.path.join(BUILD_DIR, "libsph_oracle.so")


def build(out: str = None, sanitize: bool = False) -> str:
    """Compiles the oracle; sanitize=True adds the host AddressSanitizer and
    UndefinedBehaviorSanitizer (the loading process must preload libasan)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    out = out or library_path()
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", SOURCE, "-o", tmp, "-lm"]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-g"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
