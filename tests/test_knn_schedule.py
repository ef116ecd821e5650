"""Host check of the kNN tile-pair schedules: the closed-form helpers of knn.hip are
compiled with g++ (HIP qualifiers defined away) and walked for 1 .. 300 tiles."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KNN = os.path.join(ROOT, "paper_2606_06329_amd", "csrc", "knn.hip")
MAIN = os.path.join(ROOT, "tests", "cpp", "knn_schedule_main.cpp")


def _helpers():
    src = open(KNN).read()
    start = src.index("__host__ __device__ __forceinline__ int64_t range_owner")
    end = src.index("// Cross terms D", start)
    kbq = re.search(r"constexpr int KBQ = (\d+);", src).group(1)
    return ("#include <cstdint>\n#include <cstdio>\n#include <cstdlib>\n#include <vector>\n"
            "#define __host__\n#define __device__\n#define __forceinline__ inline\n"
            f"constexpr int KBQ = {kbq};\n" + src[start:end])


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_tile_pair_schedules(tmp_path):
    cpp = tmp_path / "knn_schedule.cpp"
    cpp.write_text(_helpers() + open(MAIN).read())
    exe = tmp_path / "knn_schedule"
    subprocess.run(["g++", "-O1", "-std=c++17", str(cpp), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe), "300"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout[-2000:]
    assert "bad=0" in out.stdout
