"""The C-ABI header is plain C: it compiles as C99 and as C++17, and a C program that
calls every entry point links against the built library (nothing is run)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
LIB_DIR = os.path.join(ROOT, "paper_2009_00745_amd")

C_PROGRAM = r"""
#include <stddef.h>
#include "lise.h"
int main(void) {
    lise_ctx *c = NULL;
    lise_lattice lat = {8, 8, 8, 0, 1.0};
    lise_functional fn = {0};
    lise_obs obs;
    lise_tuning tun = {0};
    lise_batch *b = NULL;
    double g = 0.0, t = 0.0;
    int64_t s = 0, bytes = 0, n = 0;
    double ms = 0.0;
    fn.ncomp = 2;
    if (argc_guard()) {
        lise_init(&c, &lat, 4, &fn, NULL);
        lise_set_qpwf(c, 0, 1, NULL, 0);
        lise_get_qpwf(c, 0, 1, NULL, 0);
        lise_apply_h(c, 0, 1, NULL, 0);
        lise_apply_h_noalloc(c, 0, 1, NULL);
        lise_startup(c, 0.01);
        lise_step(c, 0.01, 1);
        lise_densities(c, NULL, NULL, 0);
        lise_observables(c, &obs);
        lise_get_time(c, &t, &s);
        lise_set_time(c, 0.0);
        lise_set_stream(c, NULL);
        lise_set_tuning(c, &tun);
        lise_profile(c, 1);
        lise_profile_read(c, 0, &n, &ms);
        lise_autotune(c, 0.01, 1, &tun);
        lise_memory(c, &bytes);
        lise_kick(c, NULL, 0);
        lise_current(c, NULL, 0);
        lise_save(c, "x", 1);
        lise_load(c, "x");
        lise_batch_create(&b, 1, &c, NULL);
        lise_batch_step(b, 0.01, 1);
        lise_batch_set_graph(b, 1);
        lise_batch_info(b, NULL, NULL);
        lise_batch_profile(b, 1);
        lise_batch_profile_read(b, 0, &n, &ms);
        (void)lise_batch_last_error(b);
        lise_batch_free(b);
        (void)lise_last_error(c);
        lise_free(c);
    }
    (void)lise_version();
    return lise_coupling(&lat, &fn, &g) == LISE_OK ? 0 : 1;
}
"""


def _guarded(src):
    # never executed: the calls only have to compile and link
    return "static int argc_guard(void) { return 0; }\n" + src


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_compiles_as_c99(tmp_path):
    f = tmp_path / "use.c"
    f.write_text(_guarded(C_PROGRAM))
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only", "-I", INC, str(f)], check=True)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_header_compiles_as_cpp17(tmp_path):
    f = tmp_path / "use.cpp"
    f.write_text(_guarded(C_PROGRAM))
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", "-fsyntax-only", "-I", INC, str(f)], check=True)


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.exists(os.path.join(LIB_DIR, "liblise.so")),
                    reason="gcc or the built library not available")
def test_c_program_links_against_the_library(tmp_path):
    f = tmp_path / "use.c"
    f.write_text(_guarded(C_PROGRAM))
    exe = tmp_path / "use"
    subprocess.run(["gcc", "-std=c99", "-I", INC, str(f), "-L", LIB_DIR, "-llise", "-Wl,-rpath," + LIB_DIR,
                    "-Wl,--allow-shlib-undefined", "-o", str(exe)], check=True)
    assert exe.exists()
