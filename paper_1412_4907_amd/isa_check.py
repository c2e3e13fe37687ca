"""Static check of the built gfx950 kernels for one hazard the compiler does
not cover: an instruction other than an MFMA writing a register that an
earlier MFMA reads as its accumulator input (SrcC) when that register is not
the MFMA's own destination, fewer than ``WAIT`` wait states after the MFMA.

The MFMA reads SrcC some cycles after it issues.  For the 16x16x32 FP16/BF16
MFMAs the compiler allows three wait states before such a write; rewrites
three to six wait states behind the MFMA were observed to corrupt the first
accumulator row of lanes 12-15 of each 16-lane group.  The kernels are
written so that the rewrite never comes sooner than ``WAIT`` wait states
(seven, the distance the compiler itself keeps for the 8-pass FP32 MFMA:
every MFMA is treated as that case);
this module verifies that on the assembly the build writes (hipcc
``-save-temps``).

Wait states are counted conservatively: one per instruction issued in
between (an intervening MFMA counts one), ``s_nop n`` counts n + 1.  The
scan follows fall-through across labels and conditional branches, and also
the first ``WAIT`` instructions at the target of every branch in the window.
Only VALU instructions count as writes: a load (LDS or memory) writes its
destination when its data returns, tens to hundreds of cycles after it
issues, long after the MFMA issued before it has read SrcC; the corruption
seen came from a VALU write.

``python -m paper_1412_4907_amd.isa_check <file.s>...`` prints the findings
per kernel and exits non-zero if there are any.
"""
from __future__ import annotations

import re
import sys

WAIT = 7

_RANGE = re.compile(r'^([va])\[(\d+):(\d+)\]$')
_ONE = re.compile(r'^([va])(\d+)$')


def _regs(tok: str) -> set:
    m = _RANGE.match(tok)
    if m:
        return {(m.group(1), r) for r in range(int(m.group(2)), int(m.group(3)) + 1)}
    m = _ONE.match(tok)
    if m:
        return {(m.group(1), int(m.group(2)))}
    return set()


def _writes(op: str, ops: list) -> set:
    """Vector registers a VALU instruction writes (its first operand); none
    for other instructions (see the module note on loads)."""
    if ops and op.startswith('v_') and not op.startswith('v_mfma'):
        return _regs(ops[0])
    return set()


def parse(path: str) -> dict:
    """{kernel: (instructions, label -> index)} from an assembly file; an
    instruction is (opcode, operands, source line number)."""
    kernels = {}
    name = None
    insts, labels = [], {}
    with open(path) as f:
        for ln, line in enumerate(f, 1):
            s = line.split(';', 1)[0].strip()
            if not s:
                continue
            m = re.match(r'^([A-Za-z_.$][\w.$]*):$', s)
            if m:
                lab = m.group(1)
                if not lab.startswith('.'):
                    if name is not None:
                        kernels[name] = (insts, labels)
                    name, insts, labels = lab, [], {}
                else:
                    labels[lab] = len(insts)
                continue
            if s.startswith('.') or name is None:
                continue
            parts = s.split(None, 1)
            ops = [o.strip() for o in parts[1].split(',')] if len(parts) > 1 else []
            insts.append((parts[0], ops, ln))
    if name is not None:
        kernels[name] = (insts, labels)
    return kernels


def _scan(insts, labels, start, srcc, budget, seen):
    """First write of a register in srcc reachable from instruction `start`
    within `budget` wait states: (wait states used, index) or None."""
    i, ws = start, 0
    while i < len(insts) and ws < budget:
        op, ops, _ = insts[i]
        if op == 's_nop':
            ws += int(ops[0], 0) + 1
            i += 1
            continue
        if op.startswith('v_mfma'):
            if _regs(ops[0]) & srcc:      # an MFMA rewrites it: ordered in the matrix pipe
                return None
        elif _writes(op, ops) & srcc:
            return ws, i
        if op.startswith('s_cbranch') or op == 's_branch':
            tgt = ops[0] if ops else ''
            if tgt in labels and (tgt, ws) not in seen:
                seen.add((tgt, ws))
                hit = _scan(insts, labels, labels[tgt], srcc, budget - ws - 1, seen)
                if hit is not None:
                    return ws + 1 + hit[0], hit[1]
            if op == 's_branch':
                return None
        if op in ('s_endpgm', 's_setpc_b64'):
            return None
        ws += 1
        i += 1
    return None


def check_kernel(insts, labels, wait: int = WAIT) -> list:
    """[(line of the MFMA, line of the write, wait states)] violations."""
    out = []
    for i, (op, ops, ln) in enumerate(insts):
        if not op.startswith('v_mfma') or len(ops) < 4:
            continue
        srcc, dst = _regs(ops[3]), _regs(ops[0])
        if not srcc or srcc == dst:
            continue
        hit = _scan(insts, labels, i + 1, srcc, wait, set())
        if hit is not None:
            out.append((ln, insts[hit[1]][2], hit[0]))
    return out


def check_files(paths, wait: int = WAIT) -> dict:
    """{kernel: violations} over every kernel of the given assembly files
    (only kernels with violations)."""
    bad = {}
    for p in paths:
        for name, (insts, labels) in parse(p).items():
            v = check_kernel(insts, labels, wait)
            if v:
                bad[f"{p}:{name}"] = v
    return bad


def main(argv) -> int:
    bad = check_files(argv)
    for k, v in bad.items():
        print(f"{k}: {len(v)} SrcC rewrites within {WAIT} wait states "
              f"(first: MFMA line {v[0][0]}, write line {v[0][1]}, {v[0][2]} wait states)")
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
