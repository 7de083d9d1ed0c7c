"""The C-ABI library loads and exports every symbol include/fsmmc.h declares
(no device work: these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsmmc.h")
LIB = os.path.join(ROOT, "paper_2503_17405_amd", "libfsmmc.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fsmmc_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["fsmmc_init_chains", "fsmmc_step_fsm", "fsmmc_step_synchronized",
                 "fsmmc_collect_samples"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    from paper_2503_17405_amd import fsmmc
    assert sorted(fsmmc.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_errors_without_device_work():
    from paper_2503_17405_amd import fsmmc as F
    lib = F.lib
    out = C.c_void_p()
    # NULL context / NULL out pointers are rejected before any HIP call
    assert lib.fsmmc_init_chains(None, None, None, 1, 1, 0, None, None, None, None,
                                 C.byref(out)) == F.EINVAL
    assert b"ctx" in lib.fsmmc_last_error()
    assert lib.fsmmc_step_fsm(None, 0, None) == F.EINVAL
    assert lib.fsmmc_step_synchronized(None, 1, 0, None) == F.EINVAL
    assert lib.fsmmc_collect_samples(None, 0, 1, None, 1) == F.EINVAL
    assert lib.fsmmc_job_free(None) == F.EINVAL
    assert lib.fsmmc_ctx_destroy(None) == F.EINVAL
    assert lib.fsmmc_ctx_create(0, 0, None) == F.EINVAL
    assert F.version().startswith("fsmmc")


def test_struct_layouts_match_the_binding(tmp_path):
    # sizes and field offsets of the ABI structs as a C compiler lays them out
    import subprocess
    from paper_2503_17405_amd import fsmmc as F
    structs = {"fsmmc_target_spec": F.TargetSpec, "fsmmc_sampler_spec": F.SamplerSpec,
               "fsmmc_tune": F.Tune, "fsmmc_stats": F.Stats, "fsmmc_batch_tune": F.BatchTune,
               "fsmmc_batch_counters": F.BatchCounters, "fsmmc_server_config": F.ServerConfig,
               "fsmmc_server_done": F.ServerDone, "fsmmc_server_counters": F.ServerCounters}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fsmmc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                       text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)
