#!/bin/bash
# rocprofv3 runs behind the committed summaries of the batched kernel (the
# ragged D1Q2 ensemble with S(k) sampling and the D2Q5 ensemble, each after
# its shape autotuning): kernel trace, then SQ instruction counters per
# kernel instantiation.  Run from the repository root on the GPU host as
# `bash paper_2203_01380_amd/profile_batch.sh OUTPUT_DIR`; raw output goes to OUTPUT_DIR.
set -eo pipefail
R=$(pwd)
OUT=$(mkdir -p "${1:?usage: $0 OUTPUT_DIR}" && cd "$1" && pwd)
cd /tmp
export TMPDIR=/tmp
# (two members in the batched form's plain-loop comparison: under the
# counters every launch is serialized)
B="python $R/bench.py --no-cpu-baseline --forms batched,batched_d2q5 --steps 5 --warmup 2 --loop-members 2"
echo "[profile] kernel trace"
timeout -s KILL 300 rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof_batch -o batch -- $B > $OUT/prof_batch.log 2>&1
rm -f $OUT/prof_batch/batch_kernel_trace.csv
echo "[profile] SQ counters"
timeout -s KILL 300 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_BUSY_CYCLES SQ_WAVES --output-format csv -d $OUT/pmc_batch -o sq -- $B > $OUT/pmc_batch.log 2>&1
python3 - $OUT/pmc_batch/sq_counter_collection.csv > $OUT/pmc_batch_summary.txt <<'PY'
import collections, csv, re, sys
# per kernel instantiation: dispatches and per-dispatch counter means
agg = collections.defaultdict(lambda: collections.defaultdict(float))
n = collections.Counter()
for r in csv.DictReader(open(sys.argv[1])):
    m = re.search(r'(batch_kernel<[^>]*>)', r['Kernel_Name'])
    if not m:
        continue
    agg[m.group(1)][r['Counter_Name']] += float(r['Counter_Value'])
    if r['Counter_Name'] == 'SQ_WAVES':
        n[m.group(1)] += 1
for k in sorted(agg):
    print(k, n[k], {c: '%.4g' % (v / n[k]) for c, v in sorted(agg[k].items())})
PY
rm -f $OUT/pmc_batch/sq_counter_collection.csv
cat $OUT/pmc_batch_summary.txt
echo "[profile] done"
