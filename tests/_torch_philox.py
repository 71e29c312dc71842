"""Independent Philox4x32-10: PyTorch's own source header
(ATen/core/PhiloxRNGEngine.h), compiled into a tiny helper with g++.  Used only
as a cross-check of the oracle's generator."""
import ctypes as C
import os
import subprocess
import tempfile

_SRC = r'''
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
extern "C" void torch_philox_block(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint64_t seed = (uint64_t)key[0] | ((uint64_t)key[1] << 32);
  uint64_t subseq = (uint64_t)ctr[2] | ((uint64_t)ctr[3] << 32);
  uint64_t offset = (uint64_t)ctr[0] | ((uint64_t)ctr[1] << 32);
  at::Philox4_32 eng(seed, subseq, offset);
  for (int i = 0; i < 4; ++i) out[i] = eng();
}
'''
_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    d = tempfile.mkdtemp(prefix="torch_philox_")
    src = os.path.join(d, "p.cpp")
    so = os.path.join(d, "p.so")
    with open(src, "w") as f:
        f.write(_SRC)
    subprocess.run(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-I", inc, src, "-o", so],
                   check=True, capture_output=True)
    _lib = C.CDLL(so)
    return _lib


def block(ctr, key):
    L = load()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    L.torch_philox_block(c, k, o)
    return [int(v) for v in o]
