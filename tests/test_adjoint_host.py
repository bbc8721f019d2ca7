"""The adjoint's per-pair arithmetic, FP64 instantiation, compiled for the host
from the same source as the GPU kernels (csrc/adjoint_pair.hpp, driven by
tests/host_adjoint/adjoint_f64_host.cpp the way the kernel drives it: rows
staged pre-differenced in time tiles), against the CPU oracle.

This is where the FP64 twin's gradients were once wrong on the GPU (relative
error 0.94 on UNIFORM / OMNI, 700 balls x 9 transducers, T = 450) while its
kernel spilled registers: the same arithmetic on the host agrees with the
oracle to rounding for that configuration and for time tiles that split the
pulses, so the error was not in the arithmetic.  The kernels no longer spill
(the build refuses forward or adjoint instantiations that use scratch)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from _util import PARAMS, otime, rel_l2, small_scene
from paper_2601_00551_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def host_lib(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc is not installed")
    out = str(tmp_path_factory.mktemp("adjhost") / "libadjhost.so")
    subprocess.run([HIPCC, "-O2", "-fPIC", "-shared", "-std=c++17", "--offload-host-only", "-x", "hip",
                    "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host_adjoint", "adjoint_f64_host.cpp"), "-o", out],
                   check=True, capture_output=True, text=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.host_adjoint_f64.argtypes = [ctypes.c_int64] + [P] * 5 + [ctypes.c_int] + [P] * 6 + \
        [ctypes.POINTER(_abi.SbpModel), P, ctypes.c_int, P]
    lib.host_adjoint_f64.restype = ctypes.c_int
    return lib


def host_vjp(lib, balls, arr, model, v, TT):
    b = [np.ascontiguousarray(balls[k], np.float64) for k in PARAMS]
    q = [np.ascontiguousarray(arr[k], np.float64) for k in ("qx", "qy", "qz", "nx", "ny", "nz")]
    v = np.ascontiguousarray(v, np.float64)
    g = np.zeros((5, len(b[0])))
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert lib.host_adjoint_f64(len(b[0]), *[ptr(a) for a in b], len(q[0]), *[ptr(a) for a in q],
                                ctypes.byref(model), ptr(v), TT, ptr(g)) == 0
    return {k: g[i] for i, k in enumerate(PARAMS)}


@pytest.mark.parametrize("profile,directivity,TT", [(0, 0, 451), (0, 0, 64), (1, 1, 451), (1, 1, 37)])
def test_host_build_of_the_fp64_adjoint_matches_the_oracle(host_lib, profile, directivity, TT):
    arr, balls = small_scene(91, nb=700, nd=9)        # the configuration that failed on the GPU
    T = 450
    model = _abi.SbpModel(1.5, 0.025, 0.0, 5.0, T, 1, profile, directivity, 0, 0)
    v = np.random.default_rng(4).normal(size=(9, T))
    g = host_vjp(host_lib, balls, arr, model, v, TT)
    ref = oracle.vjp(balls, arr, otime(T, profile=profile, directivity=directivity), v)
    for k in PARAMS:
        assert rel_l2(g[k], ref[k]) <= 1e-10, (k, rel_l2(g[k], ref[k]))
