"""Host memory-safety check of the MPO channel automaton: csrc/mpo.cpp is
compiled for the host with AddressSanitizer and UndefinedBehaviorSanitizer
(-Xarch_host, so no device code is instrumented) into a small driver that
builds the Hamiltonian and current MPOs of rings and open chains over the
model sizes the tests and benchmarks use (2 to 21 molecules, 0 to 4 local
modes, 0 to 2 bond modes, 2 to 11 levels) and checks the chain length and
the MPO bond widths (1 at both ends, every site's right width equal to the
next site's left width).  No GPU: build_mpo only tabulates on the host."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_13245_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "common.h"

namespace ftd {
// build_mpo never uploads; the device allocator must not be reached
void* dev_alloc(Ctx*, size_t) { std::abort(); }
void dev_free(Ctx*, void*) {}
}

int main() {
    int checked = 0;
    for (int N : {2, 3, 4, 11, 21})
        for (int per : {0, 1})
            for (int nl : {0, 1, 2})
                for (int nloc : {0, 1, 4})
                    for (int lv : {2, 3, 11}) {
                        std::vector<double> wl(nloc, 0.7), gl(nloc, 0.5), wn(nl, 0.4), gn(nl, 0.2);
                        ftd_model m{N, nloc, nl, per, lv, lv, wl.data(), gl.data(), wn.data(),
                                    gn.data(), 0.8, 1.3, 1.0};
                        if (per && N < 3) continue;   // a ring needs three molecules
                        for (int cur : {0, 1}) {
                            ftd::Mpo* mpo = ftd::build_mpo(nullptr, m, cur != 0);
                            const int bonds = per ? N : N - 1;
                            const int L = N * (1 + nloc) + bonds * nl;
                            if (mpo->L != L || (int)mpo->s.size() != L) {
                                std::printf("bad length N=%d per=%d nl=%d nloc=%d\n", N, per, nl, nloc);
                                return 1;
                            }
                            if (mpo->s[0].wl != 1 || mpo->s[L - 1].wr != 1) {
                                std::printf("bad boundary widths\n");
                                return 1;
                            }
                            for (int i = 0; i + 1 < L; ++i)
                                if (mpo->s[i].wr != mpo->s[i + 1].wl) {
                                    std::printf("width mismatch at %d\n", i);
                                    return 1;
                                }
                            delete mpo;
                            ++checked;
                        }
                    }
    std::printf("checked %d MPOs\n", checked);
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_mpo_construction_under_address_and_ub_sanitizers(tmp_path):
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "mpo_sanitized"
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           str(drv), os.path.join(CSRC, "mpo.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "checked 486 MPOs" in r.stdout, r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
