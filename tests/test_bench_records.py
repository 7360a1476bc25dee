"""The committed HBM traffic records that bench.py turns into roofline.traffic:
each parses, names its kernel and workload, and is used only for that workload
and only while the kernel sources hash to the recorded SHA-256."""
import hashlib
import json

import pytest

import bench


def _record(path):
    rec = None
    for line in open(path):
        if line.startswith("traffic-record:"):
            rec = json.loads(line.split(":", 1)[1])
    return rec


@pytest.mark.parametrize("kernel,workload", [("push_fp32r", "full_fp32r_64x64x256_ppc32_8grains"),
                                             ("push_fp64", "full_fp64_64x64x256_ppc32_8grains")])
def test_traffic_record_is_used_only_where_it_holds(kernel, workload):
    rec = _record(bench.TRAFFIC_PROFILES[kernel])
    assert rec is not None and rec["workload"] == workload
    assert rec["kernel"] == kernel.replace("fp32r", "f32r").replace("fp64", "f64")
    # one counter read per run, calibrated by the copies: FETCH_SIZE counts half
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    got = bench.traffic_per_particle_step(kernel, workload)
    if h.hexdigest() == rec["source_sha256"]:
        assert got == pytest.approx(rec["fetch_bytes_per_particle_step"] +
                                    rec["write_bytes_per_particle_step"])
        # the records' own claim: the particle record streams once each way and
        # nothing is re-read (the node bytes add about 1 B per particle-step)
        alg = 2 * bench.RECORD_BYTES[kernel[5:]]
        assert alg <= got <= 1.05 * alg
    else:
        assert got is None
    assert bench.traffic_per_particle_step(kernel, "tiny_8x8x12_ppc2") is None
    assert bench.traffic_per_particle_step("push_batch_f32r", workload) is None
