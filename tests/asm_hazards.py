"""Static check of the library's own gfx950 assembly: on every control-flow
path from an MFMA to the first v_accvgpr_read of an accumulator register it
writes, count the wait states (one per instruction, N + 1 per s_nop N).

A build in which an MFMA chain sat behind a branch read the last
accumulator row before the MFMA had written it (wrong results, no fault);
its paths had 0-2 wait states, where the compiler itself places 8-9 within a
block.  tests/test_mfma_hazards.py requires every path to have at least 8."""
import re
import collections


def min_wait_states(asm_text):
    """{kernel symbol: minimum wait states over all MFMA -> accumulator-read
    paths} (kernels without such a path are omitted)."""
    names = [n for n in re.findall(r'\n(_ZN3sbg\w+):', asm_text)
             if re.search(r'\.type\s+' + re.escape(n) + r',@function', asm_text)]
    out = {}
    for name in names:
        i = asm_text.index('\n' + name + ':') + 1
        j = asm_text.index('s_endpgm', i)
        lines = [l.split(';')[0].strip() for l in asm_text[i:j].splitlines()]
        lines = [l for l in lines if l]
        blocks = collections.OrderedDict()
        cur = '__entry'
        blocks[cur] = []
        for l in lines[1:]:
            if re.match(r'^\.LBB\w+:', l):
                cur = l[:-1]
                blocks[cur] = []
            else:
                blocks[cur].append(l)
        order = list(blocks)
        index = {b: k for k, b in enumerate(order)}

        def regs(op):
            m = re.match(r'a\[(\d+):(\d+)\]', op)
            if m:
                return set(range(int(m.group(1)), int(m.group(2)) + 1))
            m = re.match(r'a(\d+)$', op)
            return {int(m.group(1))} if m else set()

        def cost(x):
            if x.startswith('s_nop'):
                return int(x.split()[1]) + 1
            if x.startswith('s_cbranch') or x.startswith('s_branch'):
                return 0
            return 1

        kmin = None
        for b in order:
            for pi, l in enumerate(blocks[b]):
                if not l.startswith('v_mfma'):
                    continue
                dst = regs(l.split()[1].rstrip(','))
                if not dst:
                    continue
                stack = [(b, pi + 1, 0)]
                seen = {}
                while stack:
                    bb, k, ws = stack.pop()
                    if ws > 32 or seen.get((bb, k), 1 << 30) <= ws:
                        continue
                    seen[(bb, k)] = ws
                    ins = blocks[bb]
                    stop = False
                    while k < len(ins):
                        x = ins[k]
                        m = re.match(r'^s_cbranch\w*\s+(\.LBB\w+)', x)
                        if m:
                            stack.append((m.group(1), 0, ws))
                        m = re.match(r'^s_branch\s+(\.LBB\w+)', x)
                        if m:
                            stack.append((m.group(1), 0, ws))
                            stop = True
                            break
                        if x.startswith('v_accvgpr_read') and regs(x.split(',')[1].strip()) & dst:
                            kmin = ws if kmin is None else min(kmin, ws)
                            stop = True
                            break
                        if x.startswith('v_mfma') and regs(x.split()[1].rstrip(',')) & dst:
                            stop = True   # the next MFMA of the chain: interlocked in hardware
                            break
                        ws += cost(x)
                        k += 1
                    if not stop and index[bb] + 1 < len(order):
                        stack.append((order[index[bb] + 1], 0, ws))
        if kmin is not None:
            out[name] = kmin
    return out


def _vregs(op):
    m = re.match(r'v\[(\d+):(\d+)\]$', op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r'v(\d+)$', op)
    return {int(m.group(1))} if m else set()


def dpp_fma_hazards(asm_text):
    """(count, violations) for the fused v_fmac_*_dpp statements: a DPP
    source (src0) written by a VALU instruction fewer than two wait states
    before, or a label (another predecessor) fewer than two wait states before,
    is a violation.  Wait states count one per instruction and N + 1 per
    s_nop N."""
    lines = [l.split(';')[0].strip() for l in asm_text.splitlines()]
    lines = [l for l in lines if l and not l.startswith('.') or re.match(r'^\.LBB\w+:', l or '')]
    count, bad = 0, []
    for i, l in enumerate(lines):
        if not re.match(r'v_fmac_f(32|64)_dpp\s', l):
            continue
        count += 1
        ops = [o.strip() for o in l.split(None, 1)[1].split(',')]
        src = _vregs(ops[1].split()[0])
        waits = 0
        j = i - 1
        while waits < 2 and j >= 0:
            p = lines[j]
            if re.match(r'^\.LBB\w+:', p):
                bad.append((l, 'label', waits))
                break
            m = re.match(r's_nop\s+(\d+)', p)
            if m:
                waits += int(m.group(1)) + 1
            else:
                parts = p.split(None, 1)
                if parts[0].startswith('v_') and len(parts) > 1:
                    dst = _vregs(parts[1].split(',')[0].strip())
                    if dst & src:
                        bad.append((l, p, waits))
                        break
                waits += 1
            j -= 1
    return count, bad
