"""Checks on the gfx950 assembly that hipcc emits for the kernels (built here,
no GPU needed).

Barrier publication of LDS stores: in every kernel, a workgroup barrier that
follows an LDS store in straight-line code must be preceded by an
lgkmcnt(0) wait issued after that store, or another wave may read the LDS
word before the store lands.  The persistent work-list kernel once lost that
wait on its loop's back edge (the store of the next ticket), and its waves
then ran different items."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_03284_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC) and not shutil.which("hipcc"), reason="hipcc not found")


@pytest.fixture(scope="module")
def kernel_asm(tmp_path_factory):
    from paper_2305_03284_amd import build as B
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    cmd = [HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, "ddh_kernels.hip"), "-o", str(out)]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert p.returncode == 0, p.stdout[-2000:]
    return out.read_text()


def functions(asm):
    """(name, lines) of each function in the assembly."""
    out, cur = [], None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\S+):", line)
        if m:
            cur = (m.group(1), [])
            out.append(cur)
        elif cur is not None:
            cur[1].append(line)
    return out


_WAIT = re.compile(r"^\s*s_waitcnt\b.*lgkmcnt\(0\)|^\s*s_waitcnt\s+0\s*$")
_LDS_STORE = re.compile(r"^\s*ds_(write|store|add|sub|max|min|and|or|xor|inc|dec|cmpst|wrxchg)\w*\s")


def unpublished_lds_stores(lines):
    """LDS stores followed, in straight-line code, by s_barrier with no
    lgkmcnt(0) wait between them."""
    bad = []
    for k, line in enumerate(lines):
        if not re.match(r"^\s*s_barrier\b", line):
            continue
        for j in range(k - 1, -1, -1):
            t = lines[j]
            if _WAIT.search(t) or re.match(r"^\s*s_barrier\b", t):
                break
            if _LDS_STORE.match(t):
                bad.append(t.strip())
                break
    return bad


def test_scan_finds_a_planted_missing_wait():
    lines = ["\tds_write_b32 v1, v2 offset:16", "\ts_mov_b64 s[0:1], 0", "\ts_barrier"]
    assert unpublished_lds_stores(lines) == ["ds_write_b32 v1, v2 offset:16"]
    lines.insert(2, "\ts_waitcnt lgkmcnt(0)")
    assert unpublished_lds_stores(lines) == []


def test_every_barrier_publishes_the_lds_stores_before_it(kernel_asm):
    funcs = functions(kernel_asm)
    assert any("k_frame" in n for n, _ in funcs) and any("k_mstep" in n for n, _ in funcs)
    bad = {n: b for n, lines in funcs if (b := unpublished_lds_stores(lines))}
    assert not bad, bad
