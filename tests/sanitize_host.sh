#!/bin/bash
# Host-code sanitizer check (CPU only): the oracle and the library's host
# code (mesh builder, Hilbert curve, configuration checks, C ABI) built with
# AddressSanitizer and UndefinedBehaviorSanitizer (clang's, one runtime for
# both libraries), and the CPU test suite run through them.  Works on a copy
# of the repository in a temporary directory; device code is built as usual.
# Usage: bash tests/sanitize_host.sh
set -e -o pipefail
SRC=$(cd "$(dirname "$0")/.." && pwd)
D=$(mktemp -d)/repo
mkdir -p "$D"
cp -r "$SRC/oracle" "$SRC/tests" "$SRC/workloads" "$SRC/include" "$SRC/paper_2411_14631_amd" "$SRC/pytest.ini" "$D/"
rm -rf "$D/paper_2411_14631_amd/_build" "$D/paper_2411_14631_amd/libry.so" "$D/oracle/libryo.so"
LLVM=/opt/rocm/lib/llvm
SAN="-fsanitize=address,undefined -fno-sanitize-recover=undefined -fno-omit-frame-pointer -g"
# the oracle: plain C, FP64, no contraction, OpenMP (as oracle/build.py)
$LLVM/bin/clang -std=c11 -O1 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared $SAN \
    -o "$D/oracle/libryo.so" "$D/oracle/ryo.c" "$D/oracle/poisson.c" -lm
# the library: host code sanitized (each flag for the host pass only)
(cd "$D/paper_2411_14631_amd" && python - <<'PY'
import build
build.build(extra=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"])
PY
)
ASAN=$(ls $LLVM/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)
cd "$D"
ASAN_OPTIONS=detect_leaks=0:halt_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    LD_PRELOAD="$ASAN:$LLVM/lib/libomp.so" python -m pytest tests -q -m "not gpu" -x -p no:cacheprovider
