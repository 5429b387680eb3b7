"""The FLOP model bench.py reports is the device arithmetic's own operation
count: kf_device.hpp is compiled for the host with a counting number type and
the per-step counts must equal bench.py's constants."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "flops")


def _host_header(dst):
    src = open(os.path.join(ROOT, "paper_1705_02876_amd", "csrc", "kf_device.hpp")).read()
    pre = ('#include <cmath>\n#include <cstdint>\n#include "cf.hpp"\n'
           'using std::sqrt; using std::fabs; using std::atan; using std::log; using std::copysign;\n'
           'inline CF sqrt(CF x) { cnt_sqrt++; return CF::raw(std::sqrt(x.v)); }\n'
           'static inline float __frsqrt_rn(float x) { return 1.0f / std::sqrt(x); }\n')
    src = src.replace("#include <hip/hip_runtime.h>\n", pre, 1)
    src = src.replace("#define KF_DEV __device__ __forceinline__", "#define KF_DEV static inline")
    src = src.replace("__builtin_amdgcn_rsqf(x)", "1.0f / std::sqrt(x)")
    src = src.replace("__builtin_amdgcn_sqrtf(x)", "std::sqrt(x)")
    src = src.replace("a * __builtin_amdgcn_rcpf(b)", "a / b")
    src = src.replace("__builtin_amdgcn_rcpf(x)", "1.0f / x")
    src = src.replace("__builtin_amdgcn_rcp(x)", "1.0 / x")
    src = src.replace("__builtin_amdgcn_rsq(x)", "1.0 / std::sqrt(x)")
    src = src.replace("__builtin_amdgcn_logf(x)", "std::log2(x)")
    src = src.replace("__device__ __forceinline__", "static inline")
    src = src.replace("KF_DEV double copysign_t(double a, double b) { return copysign(a, b); }",
                      "KF_DEV double copysign_t(double a, double b) { return copysign(a, b); }\n"
                      "KF_DEV CF rsqrt_t(CF x) { cnt_rsqrt++; return CF::raw(1.0 / std::sqrt(x.v)); }\n"
                      "KF_DEV CF atan_t(CF x) { cnt_atan++; return CF::raw(std::atan(x.v)); }\n"
                      "KF_DEV CF log_t(CF x) { cnt_log++; return CF::raw(std::log(x.v)); }\n"
                      "KF_DEV CF sqrt_t(CF x) { cnt_sqrt++; return CF::raw(std::sqrt(x.v)); }\n"
                      "KF_DEV CF abs_t(CF x) { return CF::raw(std::fabs(x.v)); }\n"
                      "KF_DEV CF copysign_t(CF a, CF b) { return CF::raw(std::copysign(a.v, b.v)); }\n"
                      "KF_DEV CF div_t(CF a, CF b) { return a / b; }\n"
                      "KF_DEV CF rcp_pos(CF x) { return CF(1) / x; }\n"
                      "KF_DEV CF rsqrt_pos(CF x) { return CF(1) / sqrt(x); }")
    open(dst, "w").write(src)


@pytest.fixture(scope="module")
def counts(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("flops")
    shutil.copy(os.path.join(HERE, "cf.hpp"), d)
    shutil.copy(os.path.join(HERE, "count.cpp"), d)
    _host_header(os.path.join(d, "kf_device_cf.hpp"))
    exe = os.path.join(d, "count")
    subprocess.run(["g++", "-O1", "-std=c++17", "-o", exe, os.path.join(d, "count.cpp")], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        name, flop, div, trans = line.split()
        res[name] = (int(flop), int(div), int(trans))
    return res


def test_bench_flop_constants_are_the_source_counts(counts):
    sys.path.insert(0, ROOT)
    import bench
    assert bench.FLOP_PER_LAYER == counts["propagate"][0]
    assert bench.FLOP_PER_MATERIAL == counts["material"][0]
    assert bench.FLOP_PER_HIT == counts["update"][0]
    assert bench.FLOP_PER_SMOOTH_STEP == counts["smooth_step"][0]
    assert bench.BUILD_FLOP_CHI2 == counts["chi2"][0]
    assert bench.BUILD_FLOP_STEP == counts["propagate"][0] + counts["material"][0] + counts["local_pred"][0]
