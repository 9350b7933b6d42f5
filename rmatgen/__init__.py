"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Nothing in this package computes any part of the graph method. It produces:

* Philox4x32-10 random words (Salmon et al., SC'11), counter-based, so any word
  of any stream is a pure function of (seed, stream, index);
* R-MAT edge lists (Chakrabarti et al., SDM'04) with a/b/c/d = 0.57/0.19/0.19/0.05,
  self-loops kept, duplicates removed, sorted by (src, dst); the same keys come out
  of the host generator (`rmat_edges`) and the device generator (`rmat_edges_gpu`);
* derived draws: distinct vertices by rejection, FP32 uniforms, FP32 normals,
  row-normalised edge weights.

R-MAT edge k, level l (0 <= l < scale) draws word (l mod 4) of
Philox(key = seed, counter = (k_lo, k_hi, l // 4, 0)); the quadrant is 0 if the
word is below A = floor(0.57 * 2^32), 1 below A + B, 2 below A + B + C (with
B = C = floor(0.19 * 2^32)), else 3; u gains bit (q >> 1), v gains bit (q & 1).
Other draws use Philox(key = seed, counter = (b_lo, b_hi, stream, 0)), word
index w living in block b = w // 4.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_CPU_SO = os.path.join(_HERE, "librmatgen_cpu.so")
_GPU_SO = os.path.join(_HERE, "librmatgen_gpu.so")

THR_A = 57 * 2**32 // 100
THR_B = 19 * 2**32 // 100
THR_AB = THR_A + THR_B
THR_ABC = THR_AB + THR_B

HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(gpu=True):
    """Compile the host generator with gcc and (optionally) the device one with hipcc."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _CPU_SO,
                           os.path.join(_HERE, "rmat_cpu.c")])
    if gpu:
        subprocess.check_call(["hipcc", *HIP_FLAGS, "-o", _GPU_SO,
                               os.path.join(_HERE, "rmat_gpu.hip")])


_cpu_lib = None
_gpu_lib = None


def _cpu():
    global _cpu_lib
    if _cpu_lib is None:
        if not os.path.exists(_CPU_SO):
            build(gpu=False)
        lib = ctypes.CDLL(_CPU_SO)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.rmatgen_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.rmatgen_philox4x32_10.restype = None
        lib.rmatgen_philox_stream.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                              ctypes.c_int64, ctypes.c_void_p]
        lib.rmatgen_philox_stream.restype = None
        lib.rmatgen_rmat_keys.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_void_p]
        lib.rmatgen_rmat_keys.restype = None
        _cpu_lib = lib
    return _cpu_lib


def philox_block(counter, key):
    """One Philox4x32-10 block: four 32-bit counter words and two key words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in counter])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _cpu().rmatgen_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def philox_words(seed, stream, count, first=0):
    out = np.empty(int(count), dtype=np.uint32)
    if count:
        _cpu().rmatgen_philox_stream(int(seed), int(stream), int(first), int(count),
                                     out.ctypes.data)
    return out


def rmat_keys(scale, ef, seed, first=0, count=None):
    """Raw (unsorted, with duplicates) R-MAT keys u << 32 | v for edges first..first+count-1."""
    total = int(ef) << int(scale)
    if count is None:
        count = total - first
    out = np.empty(int(count), dtype=np.uint64)
    if count:
        _cpu().rmatgen_rmat_keys(int(scale), int(seed), int(first), int(count), THR_A, THR_AB,
                                 THR_ABC, out.ctypes.data)
    return out


def rmat_edges(scale, ef, seed):
    """R-MAT edge list: src, dst int32, sorted by (src, dst), duplicates removed."""
    keys = np.unique(rmat_keys(scale, ef, seed))
    src = (keys >> np.uint64(32)).astype(np.int32)
    dst = (keys & np.uint64(0xFFFFFFFF)).astype(np.int32)
    return src, dst


def _gpu():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(_GPU_SO):
            raise RuntimeError("rmatgen device generator is not built (%s)" % _GPU_SO)
        lib = ctypes.CDLL(_GPU_SO)
        lib.rmatgen_gpu_tmp_bytes.argtypes = [ctypes.c_int64, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_size_t)]
        lib.rmatgen_gpu_tmp_bytes.restype = ctypes.c_int
        lib.rmatgen_gpu_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_void_p]
        lib.rmatgen_gpu_edges.restype = ctypes.c_int
        _gpu_lib = lib
    return _gpu_lib


def rmat_edges_gpu(scale, ef, seed, device="cuda"):
    """Same edge list as rmat_edges, generated on the GPU; returns int32 torch tensors."""
    import torch
    lib = _gpu()
    count = int(ef) << int(scale)
    dev = torch.device(device)
    tmp_bytes = ctypes.c_size_t(0)
    if lib.rmatgen_gpu_tmp_bytes(count, int(scale), ctypes.byref(tmp_bytes)) != 0:
        raise RuntimeError("rmatgen_gpu_tmp_bytes failed")
    src = torch.empty(count, dtype=torch.int32, device=dev)
    dst = torch.empty(count, dtype=torch.int32, device=dev)
    m = ctypes.c_int64(0)
    with torch.cuda.device(dev):
        keys_a = torch.empty(count, dtype=torch.int64, device=dev)
        keys_b = torch.empty(count, dtype=torch.int64, device=dev)
        tmp = torch.empty(int(tmp_bytes.value), dtype=torch.uint8, device=dev)
        d_m = torch.zeros(1, dtype=torch.int64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        rc = lib.rmatgen_gpu_edges(int(scale), count, int(seed), THR_A, THR_AB, THR_ABC,
                                   keys_a.data_ptr(), keys_b.data_ptr(), tmp.data_ptr(),
                                   tmp_bytes.value, d_m.data_ptr(), src.data_ptr(),
                                   dst.data_ptr(), ctypes.byref(m), stream)
        del keys_a, keys_b, tmp, d_m
    if rc != 0:
        raise RuntimeError("rmatgen_gpu_edges failed with code %d" % rc)
    mm = int(m.value)
    return src[:mm], dst[:mm]


# ----------------------------------------------------------------------------
# Derived draws (host). Stream ids keep unrelated draws of one seed apart.
# ----------------------------------------------------------------------------
STREAM_VERTICES = 1
STREAM_UNIFORM = 2
STREAM_NORMAL = 3


def uniform_f32(seed, count, lo=0.0, hi=1.0, stream=STREAM_UNIFORM):
    """FP32 values lo + (hi - lo) * u with u = (word >> 8) * 2^-24 in [0, 1)."""
    w = philox_words(seed, stream, count)
    u = (w >> np.uint32(8)).astype(np.float64) * 2.0**-24
    return (lo + (hi - lo) * u).astype(np.float32)


def normal_f32(seed, count, stream=STREAM_NORMAL):
    """FP32 standard normals by Box-Muller from pairs of Philox words."""
    w = philox_words(seed, stream, 2 * int(count)).astype(np.float64)
    u1 = (w[0::2] + 1.0) * 2.0**-32
    u2 = w[1::2] * 2.0**-32
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.float32)


def distinct_vertices(seed, count, n, eligible=None, stream=STREAM_VERTICES):
    """`count` distinct vertex ids drawn uniformly by rejection (Lemire multiply-shift),
    skipping ids whose `eligible` entry is False."""
    count, n = int(count), int(n)
    if eligible is not None:
        if int(np.count_nonzero(eligible)) < count:
            raise ValueError("not enough eligible vertices")
    elif count > n:
        raise ValueError("count > n")
    out, seen = [], set()
    first = 0
    while len(out) < count:
        words = philox_words(seed, stream, 4096, first=first)
        first += 4096
        for r in words:
            v = (int(r) * n) >> 32
            if v in seen or (eligible is not None and not eligible[v]):
                continue
            seen.add(v)
            out.append(v)
            if len(out) == count:
                break
    return np.array(out, dtype=np.int32)


def row_normalized_weights(src, n, seed, lo=0.1, hi=1.0):
    """FP32 uniform(lo, hi) weights, one per edge, divided by the sum over the edge's
    source row (sums in FP64, result rounded to FP32)."""
    w = uniform_f32(seed, len(src), lo, hi).astype(np.float64)
    rows = np.bincount(np.asarray(src, dtype=np.int64), weights=w, minlength=int(n))
    return (w / rows[np.asarray(src, dtype=np.int64)]).astype(np.float32)
