"""Automatic FSM construction for `sample` programs with while loops, and a
C++ generator for the resulting transition function.

The procedure follows the paper's appendix ("FSM Construction Procedure for
General Programs"): a program of the grammar

    op      := identifier                    (a straight-line code block)
    simple  := op+
    while   := W{ blocks }   or   W[name]{ blocks }
    block   := simple | while
    blocks  := block+

is (1) parsed into a tree, (2) coarsened into a tree whose nodes are blocks
(consecutive ops fuse into one simple block; Alg. "Coarsening the parse
tree"), (3) turned into an FSM recursively (Alg. "FSM creation from a
coarsened parse tree"): a simple block is a one-state FSM; a sequence of
blocks joins each child's terminal state to the next child's initial state
("N"); a while block adds an empty initial state I and an empty terminal
state T with the edges enter I -> first ("E<i>"), exit last -> T ("F<i>"),
continue last -> first ("C<i>") and skip I -> T ("S<i>"); (4) every empty
state other than the machine's initial and terminal one is collapsed (Alg.
"Collapsing empty states"): its parents are joined to its children with the
conjunction of the two labels, and conjunctions that ask one loop condition
to be both true and false at the same evaluation are dropped as impossible.

Readings where the appendix's listing is garbled: the skip edge goes from
the while block's initial state to its terminal state (the listing prints
the pair reversed, which would make skipping a loop impossible, against the
text); the filter of empty states to collapse is "empty and neither initial
nor terminal"; "N" carries no condition and is dropped from conjunctions.

An edge label is the sequence of loop-condition outcomes evaluated after
the source block runs, e.g. (("F", 2), ("C", 1)): loop 2's condition is
false (leave the inner loop), then loop 1's is true (repeat the outer body).
`emit_cpp` turns the machine into a C++ transition function
`next(k, z)` that evaluates those conditions on the chain's state z in that
order.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

__all__ = ["parse", "coarsen", "build", "collapse", "make_fsm", "emit_cpp", "Fsm"]

_TOK = re.compile(r"\s*(?:(?P<wopen>W\s*(?:\[(?P<wname>[A-Za-z_]\w*)\])?\s*\{)|(?P<close>\})|"
                  r"(?P<op>[A-Za-z_][A-Za-z0-9_]*?)(?=W\s*[\[{]|[\s{}]|$))")


# ------------------------------------------------------------------ 1. parse
def _tokens(src):
    pos, out = 0, []
    src = src.strip()
    while pos < len(src):
        m = _TOK.match(src, pos)
        if not m or m.end() == pos:
            raise ValueError("cannot tokenize at %r" % src[pos:pos + 20])
        if m.group("wopen"):
            out.append(("W", m.group("wname")))
        elif m.group("close"):
            out.append(("}", None))
        else:
            out.append(("op", m.group("op")))
        pos = m.end()
        while pos < len(src) and src[pos].isspace():
            pos += 1
    return out


def parse(src):
    """Parse tree: ("blocks", [children]) with children ("op", name) and
    ("while", name_or_None, ("blocks", [...]))."""
    toks = _tokens(src)
    i = 0

    def blocks(inside):
        nonlocal i
        kids = []
        while i < len(toks):
            kind, val = toks[i]
            if kind == "op":
                kids.append(("op", val))
                i += 1
            elif kind == "W":
                i += 1
                body = blocks(True)
                if i >= len(toks) or toks[i][0] != "}":
                    raise ValueError("unclosed while block")
                i += 1
                kids.append(("while", val, body))
            else:
                if not inside:
                    raise ValueError("unbalanced '}'")
                break
        if not kids:
            raise ValueError("empty block list")
        return ("blocks", kids)

    tree = blocks(False)
    if i != len(toks):
        raise ValueError("trailing tokens")
    return tree


# --------------------------------------------------------------- 2. coarsen
def coarsen(tree):
    """Block tree: ("blocks", [...]) whose children are ("simple", [ops]) and
    ("while", number, name, [children]); loops are numbered 1, 2, ... in
    order of their opening brace."""
    counter = [0]

    def walk(kids):
        out, run = [], []
        for k in kids:
            if k[0] == "op":
                run.append(k[1])
                continue
            if run:
                out.append(("simple", run))
                run = []
            counter[0] += 1
            num = counter[0]
            out.append(("while", num, k[1] or "loop%d" % num, walk(k[2][1])))
        if run:
            out.append(("simple", run))
        return out

    return ("blocks", walk(tree[1]))


# ----------------------------------------------------------------- 3. build
@dataclass
class Fsm:
    nodes: dict = field(default_factory=dict)  # id -> ("block", ops) | ("empty", tag)
    edges: dict = field(default_factory=dict)  # (src, dst) -> label (tuple of (kind, loop))
    initial: int = 0
    terminal: int = 0
    loops: dict = field(default_factory=dict)  # loop number -> name

    def blocks(self):
        return {k: v[1] for k, v in self.nodes.items() if v[0] == "block"}

    def out(self, n):
        return {d: lab for (s, d), lab in self.edges.items() if s == n}

    def inn(self, n):
        return {s: lab for (s, d), lab in self.edges.items() if d == n}


def build(btree):
    """FSM with empty loop states from a coarsened tree."""
    f = Fsm()
    nid = [0]

    def new(kind, payload):
        nid[0] += 1
        f.nodes[nid[0]] = (kind, payload)
        return nid[0]

    def add(s, d, lab):
        if (s, d) in f.edges:
            raise ValueError("duplicate edge %s -> %s" % (s, d))
        f.edges[(s, d)] = lab

    def conv(node):
        """Returns (initial, terminal) of the sub-FSM of node."""
        if node[0] == "simple":
            n = new("block", tuple(node[1]))
            return n, n
        kids = node[1] if node[0] == "blocks" else node[3]
        parts = [conv(k) for k in kids]
        for (a, b), (c, d) in zip(parts[:-1], parts[1:]):
            add(b, c, (("N", 0),))
        if node[0] == "blocks":
            return parts[0][0], parts[-1][1]
        num, name = node[1], node[2]
        f.loops[num] = name
        I, T = new("empty", "I%d" % num), new("empty", "T%d" % num)
        add(I, parts[0][0], (("E", num),))
        add(parts[-1][1], T, (("F", num),))
        add(parts[-1][1], parts[0][0], (("C", num),))
        add(I, T, (("S", num),))
        return I, T

    f.initial, f.terminal = conv(btree)
    return f


# -------------------------------------------------------------- 4. collapse
def _join(a, b):
    lab = tuple(x for x in a + b if x[0] != "N")
    return lab if lab else (("N", 0),)


def _impossible(lab):
    """One evaluation of a loop condition cannot be both true and false:
    E_i with S_i (at entry) or C_i with F_i (after the body) in one step."""
    seen = {}
    for kind, loop in lab:
        if kind == "N":
            continue
        when = "entry" if kind in "ES" else "end"
        val = kind in "EC"
        key = (loop, when)
        if key in seen and seen[key] != val:
            return True
        seen[key] = val
    return False


def collapse(f):
    """Remove empty states that are neither initial nor terminal (and have
    no self-transition), joining their parents to their children."""
    changed = True
    while changed:
        changed = False
        for n, (kind, _) in list(f.nodes.items()):
            if kind != "empty" or n in (f.initial, f.terminal) or (n, n) in f.edges:
                continue
            parents, children = f.inn(n), f.out(n)
            for p in parents:
                del f.edges[(p, n)]
            for c in children:
                del f.edges[(n, c)]
            del f.nodes[n]
            for p, lp in parents.items():
                for c, lc in children.items():
                    lab = _join(lp, lc)
                    if _impossible(lab):
                        continue
                    if (p, c) in f.edges:
                        raise ValueError("collapsing %s would duplicate edge %s -> %s" % (n, p, c))
                    f.edges[(p, c)] = lab
            changed = True
            break
    return f


def make_fsm(src):
    """Parse, coarsen, build and collapse; the blocks are renumbered S_1..S_K
    in program order (initial block first)."""
    f = collapse(build(coarsen(parse(src))))
    order = sorted(f.nodes)  # creation order = program order of the blocks
    ren = {old: i + 1 for i, old in enumerate(order)}
    g = Fsm(nodes={ren[k]: v for k, v in f.nodes.items()},
            edges={(ren[s], ren[d]): lab for (s, d), lab in f.edges.items()},
            initial=ren[f.initial], terminal=ren[f.terminal], loops=dict(f.loops))
    return g


# ---------------------------------------------------------------- codegen
def _label_text(lab, loops):
    return " and ".join("%s(%s)" % ({"E": "enter", "S": "skip", "C": "continue", "F": "exit", "N": "next"}[k],
                                    loops.get(i, "")) if k != "N" else "next" for k, i in lab)


def emit_cpp(f, prefix, src, names=None):
    """C++ source of the FSM: an enum of the states and a transition function

        template <class Z> __host__ __device__ inline int <prefix>_next(int k, const Z& z)

    returning the state after block k has run; loop i's condition is
    z.<loop name>() (true: run / repeat the body).  The terminal block returns
    to the initial one (the next draw).  names: optional state names per
    block number (default S<k>)."""
    names = names or {}
    blocks = f.blocks()
    P = prefix.upper()
    sname = {k: "%s_%s" % (P, (names.get(k) or "S%d" % k).upper()) for k in blocks}
    lines = ["// Generated by paper_2503_17405_amd/fsmgen.py from the program", "//   " + src,
             "// (parse, coarsen, build with empty loop states, collapse; see fsmgen.py).",
             "// Do not edit: regenerate.", "#pragma once", "",
             "enum %sState : int {" % prefix.capitalize()]
    for k in sorted(blocks):
        lines.append("    %s = %d,  // %s" % (sname[k], k, " ".join(blocks[k])))
    lines.append("};")
    lines.append("")
    lines.append("template <class Z>")
    lines.append("__host__ __device__ inline int %s_next(int k, const Z& z)" % prefix)
    lines.append("{")
    lines.append("    switch (k) {")
    for k in sorted(blocks):
        outs = f.out(k)
        lines.append("    case %s:" % sname[k])
        if k == f.terminal or not outs:
            lines.append("        return %s;  // next draw" % sname[f.initial])
            continue
        lines.extend(_decision(outs, sname, f.loops, "        "))
    lines.append("    }")
    lines.append("    return %s;" % sname[f.initial])
    lines.append("}")
    return "\n".join(lines) + "\n"


def _decision(outs, sname, loops, ind):
    """Nested ifs over the labels' conditions, in evaluation order."""
    items = [(tuple(x for x in lab if x[0] != "N"), dst) for dst, lab in outs.items()]
    return _tree(items, sname, loops, ind, 0)


def _tree(items, sname, loops, ind, depth):
    done = [dst for lab, dst in items if len(lab) == depth]
    if done:
        if len(items) != 1:
            raise ValueError("ambiguous transition")
        return [ind + "return %s;" % sname[done[0]]]
    loop = {lab[depth][1] for lab, _ in items}
    if len(loop) != 1:
        raise ValueError("conditions of different loops at one decision")
    lp = loop.pop()
    yes = [(lab, d) for lab, d in items if lab[depth][0] in "EC"]
    no = [(lab, d) for lab, d in items if lab[depth][0] in "SF"]
    out = [ind + "if (z.%s()) {" % loops[lp]]
    out += _tree(yes, sname, loops, ind + "    ", depth + 1) if yes else [ind + "    return -1;"]
    out.append(ind + "} else {")
    out += _tree(no, sname, loops, ind + "    ", depth + 1) if no else [ind + "    return -1;"]
    out.append(ind + "}")
    return out


# ------------------------------------------------------------- semantics
def program_traces(src, max_decisions):
    """Every execution of the program whose loop conditions take at most
    max_decisions evaluations: (sequence of simple blocks run, sequence of
    condition outcomes as (loop, bool)).  The reference semantics that the
    FSM must reproduce."""
    btree = coarsen(parse(src))
    out = set()

    def run(kids, i, trace, dec, k):
        # continue executing kids[i:], then call k(trace, dec)
        if i == len(kids):
            k(trace, dec)
            return
        node = kids[i]
        if node[0] == "simple":
            run(kids, i + 1, trace + (tuple(node[1]),), dec, k)
            return
        num, body = node[1], node[3]

        def loop(trace, dec):
            if len(dec) >= max_decisions:
                return
            # condition false: leave the loop
            run(kids, i + 1, trace, dec + ((num, False),), k)
            # condition true: one more pass of the body, then test again
            run(body, 0, trace, dec + ((num, True),), loop)

        loop(trace, dec)

    run(btree[1], 0, (), (), lambda t, d: out.add((t, d)))
    return out


def fsm_traces(f, max_decisions):
    """Every walk of the FSM from its initial to its terminal state whose
    labels take at most max_decisions condition outcomes: (blocks run,
    outcomes), with labels read as in program_traces."""
    out = set()
    blocks = f.blocks()

    def walk(n, trace, dec):
        if len(dec) > max_decisions:
            return
        if n in blocks:
            trace = trace + (tuple(blocks[n]),)
        if n == f.terminal:
            out.add((trace, dec))
            return
        for d, lab in f.out(n).items():
            add = tuple((i, kind in "EC") for kind, i in lab if kind != "N")
            walk(d, trace, dec + add)

    walk(f.initial, (), ())
    return out
