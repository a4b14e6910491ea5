"""The ctypes structures of the binding against the C header: a small C
program compiled with the host compiler prints every field's offset and each
structure's size as the header lays them out, and the binding must agree."""
import ctypes as C
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_2109_07527_amd import crmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# numpy names of the trace record's fields and their C names
TRACE_FIELDS = [("t0", "t0"), ("t1", "t1"), ("sweep", "sweep"), ("domain", "domain"), ("colour", "colour"),
                ("trials", "trials"), ("neighbours", "neighbours"), ("own", "own"), ("staged", "staged"),
                ("hw_id", "hw_id")]
STRUCTS = [("crmc_params", crmc.crmc_params), ("crmc_cond", crmc.crmc_cond), ("crmc_obs", crmc.crmc_obs),
           ("crmc_trial_rec", crmc.crmc_trial_rec), ("crmc_tune", crmc.crmc_tune)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_binding_structures_match_the_header():
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "crmc.h"', 'int main(void) {']
    lines.append('printf("crmc_phase_trace size %zu\\n", sizeof(crmc_phase_trace));')
    for field, c_field in TRACE_FIELDS:
        lines.append('printf("crmc_phase_trace.%s %%zu\\n", offsetof(crmc_phase_trace, %s));' % (field, c_field))
    for name, cls in STRUCTS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines += ['return 0;', '}']
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.check_output([exe], text=True).split("\n")
    want = {}
    for ln in out:
        if ln.strip():
            k, v = ln.rsplit(" ", 1)
            want[k] = int(v)
    assert crmc.TRACE_DTYPE.itemsize == want["crmc_phase_trace size"]
    for field, _ in TRACE_FIELDS:
        assert crmc.TRACE_DTYPE.fields[field][1] == want["crmc_phase_trace.%s" % field], field
    for name, cls in STRUCTS:
        assert C.sizeof(cls) == want["%s size" % name], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == want["%s.%s" % (name, field)], (name, field)
