#!/bin/bash
# Builds libhdsw.so for gfx950 next to this script's package directory, and
# fails if any kernel uses scratch memory (register spills or private
# arrays): every kernel is meant to keep its state in registers and LDS.
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
out="${here}/../libhdsw.so"
flags=(-O3 -std=c++17 -fPIC --offload-arch=gfx950
       -Xclang -target-feature -Xclang -packed-fp32-ops
       -Wall -Wno-unused-result -Wno-pass-failed
       -Rpass-analysis=kernel-resource-usage)
objs=()
pids=()
logs=()
tmp="$(mktemp -d)"
trap 'rm -rf "$tmp"' EXIT
for src in kernels.hip mfma.hip big.hip noalloc.hip driver.cpp krylov.cpp api.cpp; do
  o="${tmp}/${src%.*}.o"
  hipcc "${flags[@]}" -x hip -c "${here}/${src}" -o "$o" 2> "${tmp}/${src}.log" &
  objs+=("$o")
  pids+=($!)
  logs+=("${tmp}/${src}.log")
done
fail=0
for i in "${!pids[@]}"; do
  if ! wait "${pids[$i]}"; then fail=1; fi
  # compiler messages other than the resource report
  grep -v "kernel-resource-usage\|^ *[0-9]* | \|^ *| " "${logs[$i]}" >&2 || true
done
[ "$fail" -eq 0 ] || { echo "compilation failed" >&2; exit 1; }
# kernels with scratch memory, from the resource report
spills=$(awk '/Function Name:/ {fn=$NF-0; name=$0; sub(/.*Function Name: /, "", name); sub(/ \[-Rpass.*/, "", name)}
              /ScratchSize \[bytes\/lane\]:/ {v=$0; sub(/.*: /, "", v); sub(/ \[-Rpass.*/, "", v); if (v+0 > 0) print name " scratch " v " B/lane"}' "${logs[@]}")
if [ -n "$spills" ]; then
  echo "kernels using scratch memory:" >&2
  echo "$spills" >&2
  exit 1
fi
hipcc --offload-arch=gfx950 -shared -fPIC "${objs[@]}" -o "${out}.tmp"
mv "${out}.tmp" "$out"
echo "built $out"
