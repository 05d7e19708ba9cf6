"""Seeded synthetic inputs (random walks, Gaussian mixture, noisy queries).

Shared by the CPU oracle and the GPU library's tests and benchmark: it holds
no arithmetic of the method, only the draws.  The C source (``datagen.c``) is
built into ``libdatagen.so`` next to this file with gcc.

Seeds and streams used by the workloads:
    data 2009 (stream 0), queries 786 (stream 1), noise 1 (stream 2),
    arrivals 2 (stream 3), mixture centres 3 (stream 4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "datagen.c")
CORE = os.path.join(HERE, "dg_core.h")
LIB = os.path.join(HERE, "libdatagen.so")
GPU_SRC = os.path.join(HERE, "datagen_gpu.hip")
GPU_LIB = os.path.join(HERE, "libdatagen_gpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SEED_DATA, STREAM_DATA = 2009, 0
SEED_QUERY, STREAM_QUERY = 786, 1
SEED_NOISE, STREAM_NOISE = 1, 2
SEED_ARRIVALS, STREAM_ARRIVALS = 2, 3
SEED_CENTRES, STREAM_CENTRES = 3, 4

_lib = None
_gpu_lib = None


def _stale(lib, *srcs):
    return not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(s) for s in srcs)


def build(force: bool = True) -> str:
    """Compile libdatagen.so (gcc, -O2, no FMA contraction)."""
    if force or _stale(LIB, SRC, CORE):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-pthread", SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def build_gpu(force: bool = True) -> str:
    """Compile libdatagen_gpu.so for gfx950 (hipcc, no FMA contraction)."""
    if force or _stale(GPU_LIB, GPU_SRC, CORE):
        tmp = GPU_LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               GPU_SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, GPU_LIB)
    return GPU_LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        lib = ctypes.CDLL(LIB)
        u64, u32, i64, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int32
        vp = ctypes.c_void_p
        lib.dg_philox4x32_10.argtypes = [vp, vp, vp]
        lib.dg_random_walks.argtypes = [u64, u32, u64, i64, i32, vp, ctypes.c_int]
        lib.dg_random_walks.restype = ctypes.c_int
        lib.dg_mixture_centres.argtypes = [u64, u32, i64, i32, vp]
        lib.dg_mixture.argtypes = [u64, u32, u64, i64, i32, vp, i64, ctypes.c_double, vp, ctypes.c_int]
        lib.dg_mixture.restype = ctypes.c_int
        lib.dg_add_noise.argtypes = [u64, u32, u64, i64, i32, vp, vp, vp]
        lib.dg_add_noise.restype = ctypes.c_int
        lib.dg_uniform_ints.argtypes = [u64, u32, i64, u64, vp]
        lib.dg_uniform_ints.restype = ctypes.c_int
        lib.dg_uniforms.argtypes = [u64, u32, i64, vp]
        lib.dg_uniforms.restype = ctypes.c_int
        lib.dg_gaussians.argtypes = [u64, u32, u64, i32, vp]
        _lib = lib
    return _lib


def _threads(nthreads):
    if nthreads is not None:
        return int(nthreads)
    return max(1, min(16, os.cpu_count() or 1))


def philox4x32_10(counter, key):
    """One Philox4x32-10 block: 4 x u32 counter, 2 x u32 key -> 4 x u32."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().dg_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def gaussians(seed, stream, row, n):
    out = np.zeros(n, dtype=np.float64)
    _load().dg_gaussians(seed, stream, row, n, out.ctypes.data)
    return out


def random_walks(n, length, seed=SEED_DATA, stream=STREAM_DATA, row0=0, out=None, nthreads=None):
    """Raw (not normalised) random walks, fp32 [n, length]."""
    if out is None:
        out = np.empty((n, length), dtype=np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.size == n * length
    rc = _load().dg_random_walks(seed, stream, row0, n, length, out.ctypes.data, _threads(nthreads))
    if rc != 0:
        raise RuntimeError("dg_random_walks failed")
    return out


def random_walks_into(ptr, n, length, seed=SEED_DATA, stream=STREAM_DATA, row0=0, nthreads=None):
    """Same as random_walks, written to a raw host pointer (e.g. pinned memory)."""
    rc = _load().dg_random_walks(seed, stream, row0, n, length, ctypes.c_void_p(ptr), _threads(nthreads))
    if rc != 0:
        raise RuntimeError("dg_random_walks failed")


def mixture_centres(n_centres, length, seed=SEED_CENTRES, stream=STREAM_CENTRES):
    out = np.empty((n_centres, length), dtype=np.float64)
    _load().dg_mixture_centres(seed, stream, n_centres, length, out.ctypes.data)
    return out


def mixture(n, length, centres, sigma=20.0, seed=SEED_DATA, stream=STREAM_DATA, row0=0, out=None,
            nthreads=None):
    """Gaussian-mixture rows, integers in [0, 255] stored as fp32 [n, length]."""
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    assert centres.shape[1] == length
    if out is None:
        out = np.empty((n, length), dtype=np.float32)
    rc = _load().dg_mixture(seed, stream, row0, n, length, centres.ctypes.data, centres.shape[0],
                            float(sigma), out.ctypes.data, _threads(nthreads))
    if rc != 0:
        raise RuntimeError("dg_mixture failed")
    return out


def mixture_into(ptr, n, length, centres, sigma=20.0, seed=SEED_DATA, stream=STREAM_DATA, row0=0,
                 nthreads=None):
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    rc = _load().dg_mixture(seed, stream, row0, n, length, centres.ctypes.data, centres.shape[0],
                            float(sigma), ctypes.c_void_p(ptr), _threads(nthreads))
    if rc != 0:
        raise RuntimeError("dg_mixture failed")


def add_noise(base, sigmas, seed=SEED_NOISE, stream=STREAM_NOISE, row0=0):
    """q[i] = fl32(base[i] + sigmas[i] * g_i): base rows are already z-normalised."""
    base = np.ascontiguousarray(base, dtype=np.float32)
    n, length = base.shape
    sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigmas, dtype=np.float64), (n,)))
    out = np.empty_like(base)
    rc = _load().dg_add_noise(seed, stream, row0, n, length, base.ctypes.data, sig.ctypes.data,
                              out.ctypes.data)
    if rc != 0:
        raise RuntimeError("dg_add_noise failed")
    return out


def uniform_ints(n, bound, seed, stream):
    out = np.empty(n, dtype=np.uint64)
    rc = _load().dg_uniform_ints(seed, stream, n, bound, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("dg_uniform_ints failed")
    return out.astype(np.int64)


def uniforms(n, seed, stream):
    out = np.empty(n, dtype=np.float64)
    rc = _load().dg_uniforms(seed, stream, n, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("dg_uniforms failed")
    return out


def poisson_arrivals(n, rate, seed=SEED_ARRIVALS, stream=STREAM_ARRIVALS):
    """Arrival times (s) of an open-loop Poisson process of the given rate."""
    u = uniforms(n, seed, stream)
    return np.cumsum(-np.log(u) / float(rate))


# ---- device-side generation (same values as the host functions) ----------

def _load_gpu():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(GPU_LIB):
            raise RuntimeError("libdatagen_gpu.so is not built (datagen.build_gpu())")
        lib = ctypes.CDLL(GPU_LIB)
        u64, u32, i64, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.dg_gpu_random_walks.argtypes = [vp, u64, u32, u64, i64, i32, vp]
        lib.dg_gpu_random_walks.restype = ctypes.c_int
        lib.dg_gpu_mixture.argtypes = [vp, u64, u32, u64, i64, i32, vp, i64, ctypes.c_double, vp]
        lib.dg_gpu_mixture.restype = ctypes.c_int
        _gpu_lib = lib
    return _gpu_lib


def gpu_random_walks(out, seed=SEED_DATA, stream=STREAM_DATA, row0=0):
    """Fill the fp32 CUDA tensor out[n, length] with random walks on its device."""
    import torch
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.dim() == 2
    n, length = out.shape
    rc = _load_gpu().dg_gpu_random_walks(out.data_ptr(), seed, stream, row0, n, length,
                                         torch.cuda.current_stream(out.device).cuda_stream)
    if rc != 0:
        raise RuntimeError("dg_gpu_random_walks failed: hip error %d" % rc)
    return out


def gpu_mixture(out, centres_dev, sigma=20.0, seed=SEED_DATA, stream=STREAM_DATA, row0=0):
    """Fill out[n, length] with mixture rows; centres_dev is an fp64 CUDA tensor [C, length]."""
    import torch
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and out.dim() == 2
    assert centres_dev.is_cuda and centres_dev.dtype == torch.float64 and centres_dev.is_contiguous()
    n, length = out.shape
    rc = _load_gpu().dg_gpu_mixture(out.data_ptr(), seed, stream, row0, n, length, centres_dev.data_ptr(),
                                    centres_dev.shape[0], float(sigma),
                                    torch.cuda.current_stream(out.device).cuda_stream)
    if rc != 0:
        raise RuntimeError("dg_gpu_mixture failed: hip error %d" % rc)
    return out
