#!/usr/bin/env bash
# Host sanitizer run (CPU only): builds the oracle (gcc) and the host code of
# the HIP library (hipcc, the sanitizer flags passed to the host compilation
# only) with AddressSanitizer and UndefinedBehaviorSanitizer into a temporary
# directory, then runs the CPU tests -- oracle pins, J2 pins, fixture and the
# C ABI's argument validation -- against those builds.
# Usage: oracle/check_sanitizers.sh
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
root="$(dirname "$here")"
tmp="$(mktemp -d)"
trap 'rm -rf "$tmp"' EXIT
gcc -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=undefined -fno-omit-frame-pointer \
    -ffp-contract=off -fopenmp -shared -fPIC -o "$tmp/liboracle_san.so" "$here/hrom_oracle.c" -lm
cd "$root"
python -c "
import sys; sys.path.insert(0, '.')
from paper_2306_02687_amd import build
build.build(out='$tmp/libhrom_san.so', build_dir='$tmp/obj',
            host_flags=['-fsanitize=address', '-fsanitize=undefined', '-fno-omit-frame-pointer'])
"
export ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"
export UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1"
# two runs, one sanitizer runtime each: the oracle (gcc's), the library's
# host code (clang's, the runtime of hipcc's host compiler)
HROM_ORACLE_LIB="$tmp/liboracle_san.so" \
LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
    python -m pytest tests/test_oracle_pins.py tests/test_oracle_j2.py tests/test_oracle_fixture.py \
        -q -x -p no:cacheprovider
rt="$(dirname "$(find /opt/rocm/lib/llvm/lib/clang -name 'libclang_rt.asan-x86_64.so' | head -1)")"
HROM_LIB="$tmp/libhrom_san.so" \
LD_PRELOAD="$rt/libclang_rt.asan-x86_64.so" \
    python -m pytest tests/test_abi.py -q -x -p no:cacheprovider
