"""Build-time check of the slot-layout apply kernels' hand-scheduled loads.

The slot kernels issue their factor loads from inline assembly and wait for
them with explicit ``s_waitcnt`` instructions, so the compiler does not know
that the destination registers are being written by the memory pipeline
until the matching ``; claim`` statement (an empty asm statement that takes
the registers as in/out operands, placed after the wait).  Any
compiler-generated instruction that reads or writes one of those registers
in between (a copy, a spill, a reuse as a temporary) would see or clobber a
value that is still arriving.

``check_kernel`` runs a forward may-analysis over the kernel's control-flow
graph in the device assembly: each inline-asm block is one node that adds
the destinations of its buffer loads to the in-flight set and removes the
registers it claims; every other instruction must name no in-flight
register.  ``check_file`` applies it to every kernel whose symbol contains
the given pattern.  The wait counts themselves are not checked here; the
kernels are written so that a level's registers are claimed only after a
wait that leaves just the loads of later levels outstanding.
"""

import re
import sys

_VREG = re.compile(r"\bv\[(\d+):(\d+)\]|\bv(\d+)\b")


def _vregs(text):
    out = set()
    for m in _VREG.finditer(text):
        if m.group(3) is not None:
            out.add(int(m.group(3)))
        else:
            out.update(range(int(m.group(1)), int(m.group(2)) + 1))
    return out


def kernel_bodies(asm_text, pattern):
    """{symbol: [lines]} for every function whose symbol contains pattern."""
    out, cur, name = {}, None, None
    for line in asm_text.split("\n"):
        m = re.match(r"^(_Z\S*):", line)
        if m:
            name = m.group(1)
            cur = [] if pattern in name else None
            if cur is not None:
                out[name] = cur
            continue
        if cur is not None:
            if line.strip().startswith(".Lfunc_end"):
                cur = None
                continue
            cur.append(line)
    return out


def _items(body):
    items, i = [], 0
    while i < len(body):
        t = body[i].strip()
        if t.startswith(";;#ASMSTART"):
            j, blk = i + 1, []
            while j < len(body) and not body[j].strip().startswith(";;#ASMEND"):
                blk.append(body[j].strip())
                j += 1
            items.append(("asm", blk, i))
            i = j + 1
            continue
        m = re.match(r"^(\.LBB\d+_\d+):", body[i])
        if m:
            items.append(("label", m.group(1), i))
        elif re.match(r"^; %bb\.\d+:", t):
            items.append(("label", t.split(":")[0], i))
        elif t and not t.startswith(";") and not t.startswith("."):
            items.append(("ins", t, i))
        i += 1
    return items


def _blocks(items):
    blocks = []

    def new(name):
        b = {"name": name, "items": [], "succ": [], "term": False}
        blocks.append(b)
        return b

    cur = new("entry")
    for it in items:
        if it[0] == "label":
            nb = new(it[1])
            if cur is not None and not cur["term"]:
                cur["succ"].append(nb["name"])
            cur = nb
            continue
        if cur is None:
            cur = new("after%d" % it[2])
        cur["items"].append(it)
        if it[0] != "ins":
            continue
        words = it[1].split()
        op = words[0]
        if op == "s_branch":
            cur["succ"].append(words[1])
            cur["term"] = True
            cur = None
        elif op.startswith("s_cbranch"):
            cur["succ"].append(words[1])
            nb = new("fall%d" % it[2])
            cur["succ"].append(nb["name"])
            cur["term"] = True
            cur = nb
        elif op in ("s_endpgm", "s_setpc_b64"):
            cur["term"] = True
            cur = None
    return blocks


def _transfer(block, inflight, report=None):
    s = set(inflight)
    for it in block["items"]:
        if it[0] == "asm":
            for t in it[1]:
                if t.startswith("buffer_load"):
                    s |= _vregs(t.split(None, 1)[1].split(",")[0])
                elif t.startswith("; claim"):
                    s -= _vregs(t[len("; claim"):])
            continue
        parts = it[1].split(None, 1)
        hit = _vregs(parts[1]) & s if len(parts) > 1 else set()
        if hit and report is not None:
            report.append((it[2], it[1], sorted(hit)))
    return s


def check_kernel(body):
    """(number of asm buffer loads, [(line, instruction, registers)])."""
    items = _items(body)
    blocks = _blocks(items)
    byname = {b["name"]: b for b in blocks}
    IN = {b["name"]: set() for b in blocks}
    changed = True
    while changed:
        changed = False
        for b in blocks:
            out = _transfer(b, IN[b["name"]])
            for sname in b["succ"]:
                if sname in byname and not out <= IN[sname]:
                    IN[sname] |= out
                    changed = True
    bad = []
    for b in blocks:
        _transfer(b, IN[b["name"]], bad)
    nload = sum(1 for it in items if it[0] == "asm" for t in it[1] if t.startswith("buffer_load"))
    return nload, bad


def check_file(path, pattern="k_dd_apply_slots"):
    """Raise RuntimeError naming the first violations; return the kernel count."""
    bodies = kernel_bodies(open(path).read(), pattern)
    if not bodies:
        raise RuntimeError(f"no kernel matching {pattern} in {path}")
    errors = []
    for name, body in bodies.items():
        nload, bad = check_kernel(body)
        if nload == 0:
            errors.append(f"{name}: no inline-asm loads found")
        for line, ins, regs in bad[:5]:
            errors.append(f"{name}: line {line}: '{ins}' touches in-flight v{regs}")
    if errors:
        raise RuntimeError("in-flight register check failed:\n  " + "\n  ".join(errors))
    return len(bodies)


if __name__ == "__main__":
    print(check_file(sys.argv[1], *(sys.argv[2:3] or [])), "kernels clean")
