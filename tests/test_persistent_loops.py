"""Structure of the compiled persistent rollout kernels (CPU: hipcc
cross-compiles gfx950 device code to assembly). Each persistent loop draws a
work ticket in one thread, then every wavefront passes a barrier and reads the
ticket. If the compiler nests that loop so that the barriers sit in an inner
loop the ticket draw is outside of, lanes can re-enter the barrier and read a
stale ticket while the drawing lane waits outside, and the kernel never ends
(it did so when the task layer's thread-0 stores ended the loop body and the
ticket was drawn by thread 0 as well). The test holds every barrier and the
ticket atomic of these kernels at loop depth 1 (the persistent loop
itself)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_10247_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KERNELS = ("rollout_task_kernel", "rollout_render_kernel", "rollout_rerender_kernel")


def _asm(tmp_path):
    from paper_2509_10247_amd.build import FLAGS
    out = tmp_path / "rollout.s"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "rollout.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return out.read_text()


def _depths(body):
    """(loop depth of each s_barrier, loop depth of the first global atomic)."""
    depth, bars, atomic = 0, [], None
    for line in body.split("\n"):
        m = re.match(r"^(\.LBB\d+_\d+|; %bb\.\d+):(.*)", line)
        if m:
            d = re.search(r"Depth=(\d)", m.group(2))
            depth = int(d.group(1)) if d else 0
            own = re.search(r"This (?:Inner )?Loop Header: Depth=(\d)", m.group(2))
            if own:
                depth = int(own.group(1))
            continue
        own = re.match(r"^\s+;.*This (?:Inner )?Loop Header: Depth=(\d)", line)
        if own:  # a loop header's own depth, on the comment line after its label
            depth = int(own.group(1))
            continue
        if "s_barrier" in line:
            bars.append(depth)
        if "global_atomic_add" in line and atomic is None:
            atomic = depth
    return bars, atomic


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_persistent_loops_keep_ticket_and_barriers_in_one_loop(tmp_path):
    s = _asm(tmp_path)
    names = re.findall(r"^(_ZN2da\w*(?:%s)\w*):" % "|".join(KERNELS), s, re.M)
    assert len(names) == 32, names  # 8 variants of each kernel, the render at two workgroup sizes
    for name in names:
        i = s.index(name + ":")
        body = s[i:s.index(".Lfunc_end", i)]
        bars, atomic = _depths(body)
        assert bars and all(d == 1 for d in bars), f"{name}: barrier loop depths {bars}"
        assert atomic == 1, f"{name}: ticket atomic at loop depth {atomic}"
