"""Build libchi0_devcheck.so (the device build of chi0_math.h for GPU checks) for gfx950, next to
this file, with the library's own compiler flags."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "chi0_devcheck.hip")
LIB = os.path.join(HERE, "libchi0_devcheck.so")


def build(verbose: bool = False) -> str:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_1407_3444_amd import build as B
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [B.hipcc()] + B.HIPCC_FLAGS + ["-shared", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    rc, out = B._run(cmd)
    if rc != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
