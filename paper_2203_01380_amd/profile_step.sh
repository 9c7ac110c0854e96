#!/bin/bash
# rocprofv3 runs behind the committed summaries of the headline step kernel
# (D1Q3, L = 2^24 and 2^26, uint16): kernel trace, HBM traffic (FETCH_SIZE,
# WRITE_SIZE, each scaled by a plain 768 MiB copy), SQ instruction counters,
# and the clock per dispatch after an idle start.  Run from the repository
# root on the GPU host as `bash paper_2203_01380_amd/profile_step.sh OUTPUT_DIR`;
# raw output goes to OUTPUT_DIR.
set -eo pipefail
R=$(pwd)
OUT=$(mkdir -p "${1:?usage: $0 OUTPUT_DIR}" && cd "$1" && pwd)
cd /tmp
export TMPDIR=/tmp
B="python $R/bench.py --no-cpu-baseline"
echo "[profile] kernel trace"
timeout -s KILL 300 rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof_plain -o plain -- $B --forms plain,probes --steps 200 > $OUT/prof_plain.log 2>&1
for L in 16777216 67108864; do
  echo "[profile] FETCH_SIZE L=$L"
  timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_fetch_$L -o fetch -- $B --forms plain --steps 20 --warmup 2 --copy-probe --length $L > $OUT/pmc_fetch_$L.log 2>&1
  echo "[profile] WRITE_SIZE L=$L"
  timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_write_$L -o write -- $B --forms plain --steps 20 --warmup 2 --copy-probe --length $L > $OUT/pmc_write_$L.log 2>&1
  (cd $R && python bench.py --length $L --summarize-counters $OUT/pmc_fetch_$L/fetch_counter_collection.csv $OUT/pmc_write_$L/write_counter_collection.csv)
done
echo "[profile] SQ counters"
timeout -s KILL 180 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY --output-format csv -d $OUT/pmc_sq -o sq -- $B --forms plain --steps 20 --warmup 300 > $OUT/pmc_sq.log 2>&1
(cd $R && python bench.py --summarize-sq $OUT/pmc_sq/sq_counter_collection.csv)
echo "[profile] clock per dispatch from an idle start"
timeout -s KILL 120 rocprofv3 --pmc GRBM_GUI_ACTIVE --kernel-trace --output-format csv -d $OUT/pmc_clk -o clk -- $B --forms plain --steps 300 --warmup 5 > $OUT/pmc_clk.log 2>&1
echo "[profile] done"
