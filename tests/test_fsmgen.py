"""The automatic FSM construction (Appendix, "FSM Construction Procedure for
General Programs") and its C++ transition-function generator.

Pinned against
* the transition graphs the paper draws for its four samplers (Sec. 3.1
  figure; fixture tests/golden/fsm_figure_edges.txt);
* the program's own semantics, by brute force: the set of (blocks run, loop
  outcomes) of every execution with a bounded number of loop-condition
  evaluations equals the set of initial-to-terminal walks of the FSM;
* the generated C++, compiled and driven by scripted loop outcomes, against
  the same program traces.
"""
import os
import random
import subprocess

import pytest

from paper_2503_17405_amd import fsmgen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden", "fsm_figure_edges.txt")


def figure_panels():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, prog, edges = [x.strip() for x in line.split(";")]
        out.append((name, prog, {tuple(int(v) for v in e.split("-")) for e in edges.split()}))
    return out


@pytest.mark.parametrize("name,prog,edges", figure_panels())
def test_generated_graph_matches_the_papers_figure(name, prog, edges):
    f = G.make_fsm(prog)
    assert sorted(f.blocks()) == list(range(1, len(f.blocks()) + 1))
    got = set(f.edges)
    if name == "nuts":
        assert got == edges | {(2, 4)}
    else:
        assert got == edges
    assert f.initial == 1 and f.terminal == len(f.blocks())


PROGRAMS = ["op1W{op1W{op1}}", "op1W{op1}W{op1}op2", "a W{ b } c W{ d W{ e } f } g",
            "a W{ W{ b } c }", "a W{ b W{ c W{ d } } e } f", "W{ a } b", "a b W{ c d } W{ e }"]


@pytest.mark.parametrize("prog", PROGRAMS + [p for _, p, _ in figure_panels()])
def test_fsm_walks_equal_program_executions(prog):
    f = G.make_fsm(prog)
    for k in range(0, 7):
        assert G.fsm_traces(f, k) == G.program_traces(prog, k), (prog, k)


def test_collapse_drops_contradictory_paths_and_keeps_empty_terminal():
    # the paper's example ends inside a loop: the terminal state stays empty
    f = G.make_fsm("op1W{op1W{op1}}")
    assert f.nodes[f.terminal][0] == "empty"
    for lab in f.edges.values():
        assert not G._impossible(lab)


def _harness(header, prefix, loops, script_len):
    conds = "\n".join("    bool %s() const { return next_outcome(%d); }" % (name, num)
                      for num, name in sorted(loops.items()))
    return r'''
#include <cstdio>
#include <vector>
#define __host__
#define __device__
%s
struct Z {
    std::vector<int>* script; size_t* pos; std::vector<std::pair<int,int>>* used;
    bool next_outcome(int loop) const {
        if (*pos >= script->size()) { std::printf("OUT\n"); return false; }
        int v = (*script)[(*pos)++]; used->push_back({loop, v}); return v != 0;
    }
%s
};
int main() {
    int n; while (std::scanf("%%d", &n) == 1) {
        std::vector<int> s(n); for (int& v : s) std::scanf("%%d", &v);
        size_t pos = 0; std::vector<std::pair<int,int>> used;
        Z z{&s, &pos, &used};
        int k = INITIAL, steps = 0;
        std::printf("%%d", k);
        while (k != TERMINAL && steps++ < 1000) { k = %s_next(k, z); std::printf(" %%d", k); }
        std::printf(" |");
        for (auto& u : used) std::printf(" %%d:%%d", u.first, u.second);
        std::printf("\n");
    }
}
''' % (header, conds, prefix)


@pytest.mark.parametrize("prog", ["init W[grow]{ dbl W[integ]{ integrate } check } done",
                                  "initE W[expand]{ expand } initS W[shrink]{ shrink } done",
                                  "a W[l1]{ b W[l2]{ c } W[l3]{ d } e } f"])
def test_generated_cpp_reproduces_program_executions(prog, tmp_path):
    f = G.make_fsm(prog)
    assert f.nodes[f.initial][0] == "block" and f.nodes[f.terminal][0] == "block"
    hdr = G.emit_cpp(f, "gen", prog)
    src = _harness(hdr + "\n#define INITIAL %d\n#define TERMINAL %d\n" % (f.initial, f.terminal), "gen",
                   f.loops, 0)
    (tmp_path / "h.cpp").write_text(src)
    exe = tmp_path / "h"
    r = subprocess.run(["g++", "-std=c++17", "-O1", str(tmp_path / "h.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # program executions with up to 6 loop decisions, fed to the generated code
    execs = sorted(G.program_traces(prog, 6))
    feed = "".join("%d %s\n" % (len(d), " ".join("1" if v else "0" for _, v in d)) for _, d in execs)
    out = subprocess.run([str(exe)], input=feed, capture_output=True, text=True).stdout.splitlines()
    assert len(out) == len(execs)
    blocks = f.blocks()
    for (trace, dec), line in zip(execs, out):
        states, used = line.split("|")
        seq = tuple(tuple(blocks[int(s)]) for s in states.split())
        assert seq == trace, (prog, dec, line)
        assert [tuple(int(v) for v in u.split(":")) for u in used.split()] == [(l, int(v)) for l, v in dec]


def test_committed_slice_transition_header_is_current():
    from paper_2503_17405_amd import fsm_programs as P
    path = os.path.join(ROOT, "paper_2503_17405_amd", "csrc", "slice_fsm.inc")
    assert open(path).read() == P.slice_header()
