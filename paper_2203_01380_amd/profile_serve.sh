#!/bin/bash
# rocprofv3 runs behind the committed summaries of the serving kernel: a
# kernel trace of the request streams (3 s at 200, 100 and 50 req/s), and
# SQ instruction counters of the saturated runs (64 requests of 2^20 nodes)
# beside plain lattices at the same rates.  Run from the repository root on
# the GPU host as `bash paper_2203_01380_amd/profile_serve.sh OUTPUT_DIR`; raw output goes
# to OUTPUT_DIR.
set -eo pipefail
R=$(pwd)
OUT=$(mkdir -p "${1:?usage: $0 OUTPUT_DIR}" && cd "$1" && pwd)
cd /tmp
export TMPDIR=/tmp
echo "[profile] kernel trace of the request streams"
timeout -s KILL 300 rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof_serve -o serve -- python $R/bench.py --no-cpu-baseline --forms serving --serve-seconds 3 --steps 20 --warmup 2 > $OUT/prof_serve.log 2>&1
rm -f $OUT/prof_serve/serve_kernel_trace.csv
echo "[profile] SQ counters of the saturated runs"
timeout -s KILL 600 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_SMEM SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_BUSY_CYCLES SQ_WAVES --output-format csv -d $OUT/pmc_serve -o sq -- python $R/bench.py --no-cpu-baseline --forms serving_saturated --steps 20 --warmup 2 > $OUT/pmc_serve.log 2>&1
python3 - $OUT/pmc_serve/sq_counter_collection.csv > $OUT/pmc_serve_summary.txt <<'PY'
import collections, csv, re, sys
# per kernel instantiation: dispatches and per-dispatch counter means
agg = collections.defaultdict(lambda: collections.defaultdict(float))
n = collections.Counter()
for r in csv.DictReader(open(sys.argv[1])):
    m = re.search(r'((serve|step)_kernel<[^>]*>)', r['Kernel_Name'])
    if not m:
        continue
    agg[m.group(1)][r['Counter_Name']] += float(r['Counter_Value'])
    if r['Counter_Name'] == 'SQ_WAVES':
        n[m.group(1)] += 1
for k in sorted(agg):
    print(k, n[k], {c: '%.4g' % (v / n[k]) for c, v in sorted(agg[k].items())})
PY
rm -f $OUT/pmc_serve/sq_counter_collection.csv
cat $OUT/pmc_serve_summary.txt
echo "[profile] done"
