"""The binding's ctypes structures have the C header's layout.

A C program built with the host compiler against include/hd.h prints the
size of every structure the binding mirrors and the offset of each member
the binding names; both must equal what ctypes computes, so a member added,
dropped, reordered or retyped on one side only fails here instead of
passing wrong values through the boundary.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1508_02892_amd import hd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [
    (hd.XsChannel, "hd_xs_channel"),
    (hd.IonSpecies, "hd_ion_species"),
    (hd.Params, "hd_params"),
    (hd.LaunchConfig, "hd_launch_config"),
    (hd.DeviceCtx, "hd_device_ctx"),
    (hd.MomentSet, "hd_moment_set"),
    (hd.SwarmParams, "hd_swarm_params"),
    (hd.SwarmResult, "hd_swarm_result"),
    (hd.ServerConfig, "hd_server_config"),
    (hd.ServerCounters, "hd_server_counters"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_layout_matches_header(tmp_path):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hd.h"', "int main(void) {"]
    expect = []
    for cls, name in PAIRS:
        lines.append('  printf("%%s %%zu\\n", "%s", sizeof(%s));' % (name, name))
        expect.append("%s %d" % (name, ctypes.sizeof(cls)))
        for field, *_ in cls._fields_:
            lines.append('  printf("%%s %%zu\\n", "%s.%s", offsetof(%s, %s));'
                         % (name, field, name, field))
            expect.append("%s.%s %d" % (name, field, getattr(cls, field).offset))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    assert [g for g in got if g] == expect
