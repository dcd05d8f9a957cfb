#!/bin/sh
# Builds the CPU oracle (test infrastructure) into oracle/liborc.so with gcc.
# No fused multiply-add contraction and no fast-math: the oracle's arithmetic
# is the IEEE-754 sequence its sources spell out.
set -e
here=$(cd "$(dirname "$0")" && pwd)
gcc -O2 -std=c99 -fPIC -shared -fopenmp -ffp-contract=off -fno-fast-math \
    -Wall -Wextra -Wno-unused-parameter \
    -o "$here/liborc.so" "$here/orc_math.c" "$here/orc_phys.c" "$here/orc_step.c" -lm
