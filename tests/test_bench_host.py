"""Host logic of bench.py that needs no GPU: the one-GPU guard, the source
hashes that tie a committed traffic summary to the kernel it measured, and
the format of those summaries."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_source_hash_is_stable_and_follows_the_sources():
    for kernel, files in bench.KERNEL_SOURCES.items():
        a = bench.source_sha(kernel)
        assert re.fullmatch(r"[0-9a-f]{16}", a)
        assert bench.source_sha(kernel) == a
        for f in files:
            assert os.path.exists(os.path.join(ROOT, "paper_2412_10287_amd", "csrc", f)), f
    # the two kernels share headers but not their main sources
    assert bench.source_sha("rpq::k_persistent<1>") != bench.source_sha(bench.STACKED_PASS)


def test_traffic_summaries_name_their_kernel_and_sources():
    pat = re.compile(r"kernel=(.+?) traffic_bytes_per_launch=(\d+) sources_sha256_16=([0-9a-f]{16})")
    for kernel, name in bench.TRAFFIC_FILES.items():
        text = open(os.path.join(ROOT, "profiles", name)).read()
        m = pat.search(text)
        assert m, name
        assert m.group(1) == kernel
        assert int(m.group(2)) > 0
        # the value is reported only while the sources still hash to the summary's
        got = bench.committed_traffic(kernel)
        assert got is None or got == int(m.group(2))
        if m.group(3) == bench.source_sha(kernel):
            assert got == int(m.group(2))


def test_percentile():
    assert bench.percentile([], 50) == 0.0
    assert bench.percentile([1.0, 2.0, 3.0], 50) == 2.0
    assert bench.percentile(list(range(101)), 99) == 99.0
