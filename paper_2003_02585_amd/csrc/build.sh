#!/bin/bash
# Builds libhdsw.so for gfx950 next to this script's package directory.
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
out="${here}/../libhdsw.so"
flags=(-O3 -std=c++17 -fPIC --offload-arch=gfx950
       -Xclang -target-feature -Xclang -packed-fp32-ops
       -Wall -Wno-unused-result -Wno-pass-failed)
objs=()
pids=()
tmp="$(mktemp -d)"
trap 'rm -rf "$tmp"' EXIT
for src in kernels.hip mfma.hip big.hip driver.cpp krylov.cpp api.cpp; do
  o="${tmp}/${src%.*}.o"
  hipcc "${flags[@]}" -x hip -c "${here}/${src}" -o "$o" &
  objs+=("$o")
  pids+=($!)
done
for p in "${pids[@]}"; do wait "$p"; done
hipcc --offload-arch=gfx950 -shared -fPIC "${objs[@]}" -o "${out}.tmp"
mv "${out}.tmp" "$out"
echo "built $out"
