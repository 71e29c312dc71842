"""Independent Philox4x32-10: rocRAND's source header
(rocrand/rocrand_philox4x32_10.h), compiled with hipcc into a tiny host helper
that calls the engine's ten rounds on a given counter and key.  Used only as a
cross-check of the oracle's generator."""
import ctypes as C
import os
import subprocess
import tempfile

_SRC = r'''
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>
struct Rounds : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
extern "C" void rocrand_philox_block(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    Rounds e;
    const uint4 r = e.block(uint4{ctr[0], ctr[1], ctr[2], ctr[3]}, uint2{key[0], key[1]});
    out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
}
'''
_lib = None
HIPCC = "/opt/rocm/bin/hipcc"


def load():
    global _lib
    if _lib is not None:
        return _lib
    d = tempfile.mkdtemp(prefix="rocrand_philox_")
    src = os.path.join(d, "p.cpp")
    so = os.path.join(d, "p.so")
    with open(src, "w") as f:
        f.write(_SRC)
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-shared", "-fPIC", "--offload-arch=gfx950", src,
                    "-o", so], check=True, capture_output=True)
    _lib = C.CDLL(so)
    return _lib


def block(ctr, key):
    L = load()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    L.rocrand_philox_block(c, k, o)
    return [int(v) for v in o]
