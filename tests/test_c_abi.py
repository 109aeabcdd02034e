"""The boundary is a plain C ABI: include/qst.h compiles as strict C99 and a C program links
against libqst.so and calls it (validation-only handle: no GPU needed)."""
import os
import shutil
import subprocess

import pytest

from paper_2607_19577_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "qst.h"
int main(void) {
  qst_handle* h = NULL;
  if (qst_create(-1, NULL, &h) != QST_OK || !h) return 1;
  qst_instance in;
  memset(&in, 0, sizeof in);
  in.n_qubits = 0;
  in.rank = 1;
  in.n_settings = 1;
  in.atoms = (const void*)0x1000;
  in.weights = (const double*)0x2000;
  in.settings = (const uint8_t*)0x3000;
  qst_status s = qst_forward(h, &in, 1, NULL, NULL, QST_LOSS_NONE, 0.0, QST_PATH_AUTO);
  printf("%d|%s|%s\n", (int)s, qst_status_string(s), qst_last_error(h));
  in.n_qubits = 10;
  qst_status t = qst_forward(h, &in, 1, NULL, NULL, QST_LOSS_NONE, 0.0, QST_PATH_AUTO);
  printf("%d\n", (int)t);
  return qst_destroy(h) == QST_OK ? 0 : 2;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_program_links_and_calls_the_library(tmp_path):
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libqst.so is not built (run __graft_entry__.build())")
    src = tmp_path / "t.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "t"
    libdir = os.path.dirname(_lib.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), str(src), "-L", libdir, "-lqst", f"-Wl,-rpath,{libdir}",
                        "-o", str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    first, second = out.stdout.strip().splitlines()
    code, _, msg = first.split("|")
    assert int(code) == 2 and "n_qubits" in msg  # QST_ERR_SHAPE with the handle's message
    assert int(second) == 4  # valid arguments on a validation-only handle
