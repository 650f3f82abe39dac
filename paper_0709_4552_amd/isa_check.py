"""Build-time check of the compiled kernels: no barrier inside a divergent loop.

A workgroup barrier must be reached by every wave the same number of times.
If the compiler lowers a loop that contains s_barrier as divergent (its exit
or back-edge taken per lane under an exec mask), lanes of one wave can reach
the barrier on different trips and the workgroup can deadlock.  The lowering
of such a loop leaves, in a block whose innermost loop is that loop,
    s_andn2_b64 exec, exec, sX ; s_cbranch_exec[n]z ...
This module reads the gfx950 assembly of the library and reports every loop
that holds both that pattern and a barrier (directly or in a child loop).
"""
import re
import sys


def check_asm(text: str):
    """Return [(kernel, [loop headers])] for every offending kernel."""
    out = []
    s = text
    for m in re.finditer(r'\n(_Z\S+):\s*;.*?\n(.*?)\.Lfunc_end', s, re.S):
        name, body = m.group(1), m.group(2)
        lines = body.split('\n')
        blocks = []  # (label, innermost header or None, [instr])
        parent = {}
        cur = None
        k = 0
        while k < len(lines):
            l = lines[k]
            mm = re.match(r'^\.LBB(\d+_\d+):(.*)', l)
            mm2 = re.match(r'^; %bb\.\d+:(.*)', l)
            if mm or mm2:
                lab = mm.group(1) if mm else None
                ann = (mm.group(2) if mm else mm2.group(1))
                j = k + 1
                while j < len(lines) and lines[j].strip().startswith(';'):
                    ann += lines[j]
                    j += 1
                inner = None
                if lab and 'Loop Header' in ann:
                    inner = lab
                    ps = re.findall(r'Parent Loop BB(\d+_\d+)', ann)
                    parent[lab] = ps[-1] if ps else None
                else:
                    hs = re.findall(r'Header=BB(\d+_\d+)', ann)
                    inner = hs[-1] if hs else None
                cur = [lab, inner, []]
                blocks.append(cur)
                k = j
                continue
            if cur is not None and l.strip() and not l.strip().startswith(';'):
                cur[2].append(l.strip())
            k += 1
        def chain(h):
            out = []
            while h:
                out.append(h)
                h = parent.get(h)
            return out
        has_bar = set()
        div = set()
        for lab, inner, ins in blocks:
            if inner is None:
                continue
            if any(x.startswith('s_barrier') for x in ins):
                has_bar.update(chain(inner))
            for q in range(len(ins) - 1):
                if ins[q].startswith('s_andn2_b64 exec, exec') and ins[q + 1].startswith('s_cbranch_exec'):
                    div.add(inner)
        bad = sorted(div & has_bar)
        if bad:
            out.append((name, bad))
    return out


def count_kernels(text: str) -> int:
    return len(re.findall(r'\n(_Z\S+):\s*;', text))


if __name__ == "__main__":
    worst = 0
    for fn in sys.argv[1:]:
        res = check_asm(open(fn).read())
        for name, bad in res:
            print("divergent barrier loop:", name, bad)
        worst |= bool(res)
    sys.exit(1 if worst else 0)
