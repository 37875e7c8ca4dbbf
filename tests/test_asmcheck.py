"""The in-flight register check of the hand-scheduled apply loads: it passes
clean code, catches a read or a spill of a register between its load and its
claim (also across a loop's back edge and in blocks placed out of line), and
the device assembly of the shipped apply kernels passes it."""

import os
import subprocess

import pytest

from paper_2508_04917_amd import asmcheck
from paper_2508_04917_amd import build as B

LOAD = """\t;;#ASMSTART
\tbuffer_load_dwordx4 v[2:5], v1, s[0:3], 0 offen offset:16
\t;;#ASMEND
"""
WAIT = """\t;;#ASMSTART
\ts_waitcnt vmcnt(0)
\t;;#ASMEND
"""
CLAIM = """\t;;#ASMSTART
\t; claim v[2:5]
\t;;#ASMEND
"""


def kernel(body):
    return "_Z1kv:\n" + body + "\ts_endpgm\n.Lfunc_end0:\n"


def check(text):
    bodies = asmcheck.kernel_bodies(text, "_Z1kv")
    assert len(bodies) == 1
    return asmcheck.check_kernel(next(iter(bodies.values())))


def test_straight_line_clean():
    nload, bad = check(kernel(LOAD + "\tv_mov_b32 v6, v7\n" + WAIT + CLAIM + "\tv_add_f32 v8, v2, v3\n"))
    assert nload == 1 and bad == []


def test_read_before_claim():
    nload, bad = check(kernel(LOAD + "\tv_mov_b32 v9, v3\n" + WAIT + CLAIM))
    assert [b[2] for b in bad] == [[3]]


def test_spill_before_claim():
    spill = "\tscratch_store_dwordx4 off, v[4:7], off ; 16-byte Folded Spill\n"
    nload, bad = check(kernel(LOAD + spill + WAIT + CLAIM))
    assert [b[2] for b in bad] == [[4, 5]]


def test_write_before_claim():
    nload, bad = check(kernel(LOAD + "\tv_mov_b32 v5, 0\n" + WAIT + CLAIM))
    assert [b[2] for b in bad] == [[5]]


def loop(top):
    # the load at the bottom of the body is claimed at the top of the next pass
    return kernel(
        ".LBB0_1:\n" + top + CLAIM + "\tv_add_f32 v8, v2, v3\n" + LOAD
        + "\ts_cmp_lt_i32 s4, s5\n\ts_cbranch_scc1 .LBB0_1\n")


def test_loop_back_edge():
    assert check(loop(WAIT))[1] == []
    bad = check(loop(WAIT + "\tv_mul_f32 v9, v2, v2\n"))[1]
    assert [b[2] for b in bad] == [[2]]


def test_out_of_line_block():
    # the fetch block sits after the end of the program and jumps back
    text = kernel(
        "\ts_cmp_eq_u32 s4, 0\n\ts_cbranch_scc0 .LBB0_3\n.LBB0_2:\n" + WAIT
        + "\tv_mov_b32 v9, v4\n" + CLAIM + "\tv_add_f32 v8, v2, v3\n\ts_endpgm\n.LBB0_3:\n" + LOAD
        + "\ts_branch .LBB0_2\n")
    bad = check(text)[1]
    assert [b[2] for b in bad] == [[4]]


def test_no_loads_is_an_error(tmp_path):
    p = tmp_path / "a.s"
    p.write_text(kernel("\tv_mov_b32 v1, v2\n").replace("_Z1kv", "_Z16k_dd_apply_slotsv"))
    with pytest.raises(RuntimeError, match="no inline-asm loads"):
        asmcheck.check_file(str(p))


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not available")
def test_shipped_apply_kernels(tmp_path):
    """Device assembly of apply.hip, built with the library's flags."""
    out = tmp_path / "apply.s"
    subprocess.run([B.HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(B.CSRC, "apply.hip"),
                    "-o", str(out)], check=True, stderr=subprocess.DEVNULL, cwd=tmp_path)
    n = asmcheck.check_file(str(out))
    assert n >= 100  # every (block size, precision, threads, slots, depth, correction) instance
