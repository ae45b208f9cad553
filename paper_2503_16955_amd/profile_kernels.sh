#!/bin/bash
# rocprofv3 runs behind profiles/: the kernel trace of the benchmark's trace
# kernels, the kernel trace of a serving run, that of the extended-input
# kernels, HBM byte counters of the trace
# kernels and of a plain 256 MiB copy (the scale reference), SQ
# instruction and lane-activity counters and the detector's atomics; then
# the VALU issue-rate microbenchmark
# (valu_rates, built by build.py) behind the roofline's slot weights.  Each pass is a run of its own (counters are not
# multiplexed).  Usage: profile_kernels.sh OUT_DIR   (run from anywhere)
set -u
R=$(cd "$(dirname "$0")/.." && pwd)
OUT=$(mkdir -p "$1" && cd "$1" && pwd)
export TMPDIR=/tmp PYTHONPATH=$R
cd /tmp
B="python3 $R/bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-serving --shard-of 0 --no-extended --no-stress --no-burn-in"
B1="python3 $R/bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-serving --shard-of 0 --no-extended --no-stress --no-burn-in"
S="python3 $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-mixed --serving-requests 64 --shard-of 0 --no-extended --no-stress --no-mwg"
E="python3 $R/bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-serving --no-mwg --shard-of 0 --no-stress --no-burn-in"
C="python3 -m paper_2503_16955_amd.profiling copy --mib 256"
step() {   # name, time limit (s), command...
    local name=$1 lim=$2; shift 2
    echo "== $name $(date +%T)"
    timeout -k 10 "$lim" "$@" > "$OUT/prof_$name.log" 2>&1
    local rc=$?
    echo "$name rc=$rc"
    # rocprofv3 itself may end with SIGSEGV (139) after the profiled program
    # has finished; that counts only when the program's own last line (the
    # bench's JSON line, the copy's byte count) is in its log
    if [ $rc -eq 139 ] && tail -n 3 "$OUT/prof_$name.log" | grep -q -e '"metric"' -e '^copied '; then
        echo "$name: profiler ended with 139 after a complete run"
        rc=0
    fi
    if [ $rc -ne 0 ]; then exit $rc; fi
}
step trace 240 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/prof_trace" -o trace -- $B
step serve 240 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/prof_serve" -o serve -- $S
step ext 240 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/prof_ext" -o ext -- $E
step fetch 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d "$OUT/prof_fetch" -o fetch -- $B1
step write 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d "$OUT/prof_write" -o write -- $B1
step cfetch 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d "$OUT/prof_cfetch" -o cfetch -- $C
step cwrite 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d "$OUT/prof_cwrite" -o cwrite -- $C
step sq1 120 rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_SMEM SQ_INSTS_LDS SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES --output-format csv -d "$OUT/prof_sq1" -o sq1 -- $B1
step sq2 120 rocprofv3 --pmc SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_CVT SQ_INSTS_VALU_TRANS_F32 --output-format csv -d "$OUT/prof_sq2" -o sq2 -- $B1
step sq3 120 rocprofv3 --pmc SQ_THREAD_CYCLES_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_FMA_F32 SQ_INSTS_BRANCH SQ_WAIT_INST_ANY SQ_INSTS_VSKIPPED --output-format csv -d "$OUT/prof_sq3" -o sq3 -- $B1
step atom 120 rocprofv3 --pmc TCC_ATOMIC_sum TCC_EA0_ATOMIC_sum TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum TA_FLAT_ATOMIC_WAVEFRONTS_sum --output-format csv -d "$OUT/prof_atom" -o atom -- $B1
echo "== valu_rates $(date +%T)"
timeout -k 10 120 "$R/paper_2503_16955_amd/valu_rates" > "$OUT/valu_rates.md" 2>&1 || exit $?
echo "done $(date +%T)"
