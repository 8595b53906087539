#!/bin/bash
# The CPU test suite with the FP64 oracle, the scene generator and the host
# code of the HIP library built with AddressSanitizer and UBSan (clang), the
# sanitizers' runtime preloaded into Python.  Device code is built as usual
# and never runs here.  Extra arguments go to pytest.
#
#   bash tests/run_cpu_sanitized.sh [-x] [-k pattern]
set -euo pipefail
ROOT="$(cd "$(dirname "${BASH_SOURCE[0]}")/.." && pwd)"
cd "$ROOT"
export UPS_SANITIZE=1
python -m paper_2101_00585_amd.build --sanitize > /dev/null
python -c "import oracle, synth; oracle.build(); synth.build()"
RT="$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so)"
# leaks: Python and the HIP runtime keep allocations until exit by design
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 LD_PRELOAD="$RT" \
    python -m pytest tests -m "not gpu" -q -p no:cacheprovider "$@"
