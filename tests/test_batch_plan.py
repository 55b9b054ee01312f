"""Host-side checks of the batched sweeps' descriptor tables, without a GPU.

tests/batch_plan_check.cpp is compiled here with the host compiler against the
library's planner (paper_2401_15758_amd/csrc/batch_plan.hpp).  For the batch-64
problems and every tiling of the batched tiling search it bounds every index
the batched FWD / TLM / ADJ kernels derive from the staged tables, checks that
the tiles partition each grid, and that every staged group fits half of the
staging ring.  It also replays the ring placement of a batched FWD followed by
a block Hessian's sweeps under the earlier policy (drain and restart at 0 when
a table does not fit) and the current one: the earlier policy overwrites the
argument blocks of a sweep with its own work items for tilings whose item
table exceeds half the ring, the current one never overwrites a table of its
own group."""
import os
import shutil
import subprocess

import pytest

from paper_2401_15758_amd import autotune, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "batch_plan_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("plan") / "batch_plan_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2401_15758_amd", "csrc"), SRC, "-o", exe], check=True)
    return exe


def _run(exe, cfgs, tilings, ks):
    lines = [str(len(cfgs))]
    lines += [f"{c['n']} {c['nsteps']} {c['obs_stride']} {c['obs_every']}" for c in cfgs]
    lines.append(str(len(tilings)))
    lines += [f"{t['xch']} {t['ppt']} {t['kc']} {t['threads']} {t['steps']}" for t in tilings]
    lines.append(str(len(ks)))
    lines.append(" ".join(str(k) for k in ks))
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout


def test_batch64_tables_in_bounds_for_every_searched_tiling(checker):
    cfgs = inputs.batch_configs(64, seed=0)
    tilings = autotune.batch_candidates()
    rc, out = _run(checker, cfgs, tilings, [32, 1])
    last = out.strip().splitlines()[-1]
    assert rc == 0, out[-4000:]
    assert last.startswith("planned") and last.endswith("violations 0"), last
    planned = int(last.split()[1])
    assert planned == 2 * len(tilings)          # every tiling plans for k = 32 and k = 1
    assert " new_overwrites 0 " in last


def test_earlier_ring_policy_overwrote_sweep_tables(checker):
    """Item tables between half and all of the 32 MiB ring (small regions, few
    vectors per group): replayed from each 1 MiB starting offset of the ring,
    the earlier policy -- drain and restart at 0 when a table does not fit --
    stages a sweep's items over its own argument blocks for some starts, which
    hands the kernels argument blocks made of work items: wild pointers.  The
    default tiling's tables never reach that size, and the current placement
    (chunked groups within one half) never overwrites a table of its group."""
    cfgs = inputs.batch_configs(64, seed=0)
    tilings = [dict(xch=2, ppt=2, kc=2, threads=256, steps=12), dict(xch=1, ppt=1, kc=1, threads=256, steps=4),
               dict(xch=2, ppt=4, kc=2, threads=256, steps=12)]
    rc, out = _run(checker, cfgs, tilings, [32])
    assert rc == 0, out[-4000:]
    rows = [l.split() for l in out.splitlines() if l.startswith("xch")]
    old = {tuple(r[:5]): int(r[r.index("old_overwrites") + 1]) for r in rows}
    new = {tuple(r[:5]): int(r[r.index("new_overwrites") + 1]) for r in rows}
    assert old[("xch2", "ppt2", "kc2", "thr256", "S12")] > 0
    assert old[("xch1", "ppt1", "kc1", "thr256", "S4")] > 0
    assert old[("xch2", "ppt4", "kc2", "thr256", "S12")] == 0       # the default tiling
    assert len(new) == 3 and all(v == 0 for v in new.values())


def test_ring_group_placement():
    """The two-halves placement on its own: a group goes to the other half (after
    a drain) when it does not fit in the rest of the current one, never
    straddles the halves, and a group larger than a half is refused."""
    import ctypes  # noqa: F401  (pure arithmetic, mirrored from batch_plan.hpp by the checker build)
    cap = 1024
    half = cap // 2

    def place(off, nbytes):
        base = 0 if off < half else half
        if nbytes > half:
            return None
        if off + nbytes > base + half:
            first = half if base == 0 else 0
            return first, first + nbytes, True
        return off, off + nbytes, False

    assert place(0, 512) == (0, 512, False)
    assert place(256, 512) == (512, 1024, True)
    assert place(768, 256) == (768, 1024, False)
    assert place(800, 256) == (0, 256, True)
    assert place(0, 513) is None


@pytest.fixture(scope="module")
def checker_sanitized(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("plan_san") / "batch_plan_check_san")
    r = subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2401_15758_amd", "csrc"), SRC, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("host sanitizer runtime not available")
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_planner_under_address_and_undefined_behaviour_sanitizers(checker_sanitized):
    """The host planner and ring placement (the library's own header code) built
    with AddressSanitizer and UndefinedBehaviorSanitizer, on a sample of the
    batch-64 problems and of the searched tilings: no sanitizer report, and the
    same verdicts as the plain build."""
    cfgs = inputs.batch_configs(64, seed=0)[::4]
    tilings = autotune.batch_candidates()[::9]
    rc, out = _run(checker_sanitized, cfgs, tilings, [32, 1])
    last = out.strip().splitlines()[-1]
    assert rc == 0, out[-4000:]
    assert last.startswith("planned") and last.endswith("violations 0"), last
