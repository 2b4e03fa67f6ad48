#!/bin/bash
# Builds the library's host code with a sanitizer and links the mesh set-up
# driver against it: ./build.sh address|thread <output dir>.  Device code is
# compiled as usual (the sanitizer flag goes to the host pass only); nothing
# here runs on a GPU.
set -e
SAN=${1:-address}
OUT=${2:-$(dirname "$0")/../../_build/sanitize-$SAN}
HERE=$(cd "$(dirname "$0")" && pwd)
R=$(cd "$HERE/../.." && pwd)
mkdir -p "$OUT"
INC="-I$R/include -I$R/paper_2305_15116_amd/csrc"
pids=()
for f in "$R"/paper_2305_15116_amd/csrc/*.hip; do
  b=$(basename "$f" .hip)
  /opt/rocm/bin/hipcc -x hip --offload-arch=gfx950 -O1 -g -std=c++17 -fPIC $INC -Xclang -target-feature -Xclang -packed-fp32-ops \
    -Xarch_host -fsanitize=$SAN -Xarch_host -fno-omit-frame-pointer -c "$f" -o "$OUT/$b.o" 2>/dev/null &
  pids+=($!)
done
for f in "$R"/paper_2305_15116_amd/csrc/*.cpp "$HERE"/mesh_setup_driver.cpp; do
  b=$(basename "$f" .cpp)
  g++ -O1 -g -std=c++17 -fPIC -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include $INC -fsanitize=$SAN -fno-omit-frame-pointer \
    -c "$f" -o "$OUT/$b.o" &
  pids+=($!)
done
for p in "${pids[@]}"; do wait "$p"; done
/opt/rocm/bin/hipcc --offload-arch=gfx950 -Xarch_host -fsanitize=$SAN "$OUT"/*.o -o "$OUT/mesh_setup_driver" -lpthread
echo "$OUT/mesh_setup_driver"
