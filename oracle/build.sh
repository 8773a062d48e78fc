#!/bin/sh
# Builds the FP64 CPU oracle (test infrastructure) as oracle/liboracle.so.
set -e
cd "$(dirname "$0")"
gcc -O2 -std=c11 -Wall -fopenmp -fPIC -shared -o liboracle.so rve.c sparse.c macro.c -lm
