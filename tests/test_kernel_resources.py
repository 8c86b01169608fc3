"""Register use and occupancy of the hot kernels, from the compiler's resource report.

The traversal is latency bound: each wave per SIMD it loses costs far more than the
few instructions that caused it (a guard of two compares once took the batched
traversal from 109 to 136 VGPRs, 4 to 3 waves per SIMD, and 40% more time).  This
compiles the sources for gfx950 (device code only, no GPU needed) and checks each
hot kernel against the occupancy and scratch it is designed for.
"""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_00444_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")

# kernel-name pattern -> (minimum waves per SIMD, maximum scratch bytes per lane)
EXPECT = {
    "query.hip": {
        r"traverse_batch_kernelILb1ELi(2|4|8|16|32)ELi4EE": (4, 0),
        # the five-wave variant for launches beyond four waves per SIMD: its few
        # spills (24 B) sit outside the round loop
        r"traverse_batch_kernelILb1ELi(2|4|8|16|32)ELi5EE": (5, 32),
        r"traverse_batch_kernelILb0ELi(16|32)ELi4EE": (6, 0),
    },
    "lbvh.hip": {
        # three 512-thread workgroups per CU: 6 waves per SIMD
        r"refit_kernelILb1ELi512ELi[12]ELi6EE": (6, 0),
        r"frame_update_kernelILi512ELi[12]ELi6EE": (6, 0),
        r"radix_pass_kernelILi2EE": (8, 0),
        r"hierarchy_kernel": (8, 0),
        r"morton_kernel": (8, 0),
    },
}


def _report(src):
    cmd = [HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           "--cuda-device-only", "-c", os.path.join(CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def _parse(text):
    """{mangled name: {'vgpr': int, 'scratch': int, 'waves': int}} from the remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        if cur is None:
            continue
        for key, pat in (("vgpr", r"remark:\s+VGPRs: (\d+)"), ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("waves", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m:
                cur[key] = int(m.group(1))
    return out


@pytest.mark.skipif(HIPCC is None, reason="hipcc not installed")
def test_hot_kernels_keep_their_occupancy():
    procs = {src: _report(src) for src in EXPECT}
    problems = []
    for src, proc in procs.items():
        text, _ = proc.communicate(timeout=600)
        assert proc.returncode == 0, text[-2000:]
        kernels = _parse(text)
        for pat, (waves, scratch) in EXPECT[src].items():
            hits = {k: v for k, v in kernels.items() if re.search(pat, k)}
            assert hits, f"{src}: no kernel matches {pat}"
            for name, r in hits.items():
                if r.get("waves", 0) < waves or r.get("scratch", 1 << 30) > scratch:
                    problems.append(f"{name}: {r} (want >= {waves} waves/SIMD, <= {scratch} B scratch)")
    assert not problems, "\n".join(problems)
