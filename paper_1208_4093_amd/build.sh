#!/bin/bash
# Build libtl.so for gfx950 in-tree.  Packed-FP32 instructions are disabled on
# purpose (some of their forms have produced wrong results on these GPUs).
set -euo pipefail
HERE="$(cd "$(dirname "${BASH_SOURCE[0]}")" && pwd)"
ROOT="$(dirname "$HERE")"
OUT="$HERE/libtl.so"
FLAGS=(--offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared
       -Xclang -target-feature -Xclang -packed-fp32-ops
       -I"$ROOT/include" -I"$HERE/csrc")
/opt/rocm/bin/hipcc "${FLAGS[@]}" "$HERE/csrc/tl_kernels.hip" "$HERE/csrc/tl_host.cpp" "$HERE/csrc/tl_batch.cpp" "$HERE/csrc/tl_noalloc.hip" "$HERE/csrc/tl_tune.cpp" -o "$OUT.tmp"
mv "$OUT.tmp" "$OUT"
echo "built $OUT"
