"""Host-side pieces of bench.py: the algorithmic-byte count the roofline is
stated on, and the lookup of stored HBM counters, which must answer only for
the operation, batch, plan and kernel the counters were taken on."""
from types import SimpleNamespace

import bench


def test_keyswitch_algorithmic_bytes():
    # (4, 2^16, 32): k = alpha = 8, 4 digits, 40 limbs with P; d + out + evk / B
    G = SimpleNamespace(n=1 << 16, ell=32, ndig=4, nl=40)
    W = 8
    assert bench.ks_algorithmic_bytes(G, 8) == 32 * G.n * W + 2 * 32 * G.n * W + 4 * 2 * 40 * G.n * W / 8
    assert bench.ks_algorithmic_bytes(G, 8) == 71303168  # 71.3 MB per KeySwitch at batch 8
    # the key's share shrinks with the batch, the ciphertext's does not
    assert bench.ks_algorithmic_bytes(G, 1) - bench.ks_algorithmic_bytes(G, 8) == 4 * 2 * 40 * G.n * W * (1 - 1 / 8)


def test_stored_traffic_answers_only_its_own_measurement():
    t = bench.TRAFFIC
    args = (t["workload"], t["op"], t["batch"], t["plan"], t["kernel"])
    got = bench.measured_traffic(*args)
    if t["sources_sha256"] == bench.kernel_sources_sha256():
        assert got == int((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)
    else:  # kernels changed since the counters were taken
        assert got is None
    for i, other in enumerate(("d2-n13-l6", "hmul", t["batch"] // 2, "Plan(STAGED, chunks=1, log_r=4, mfma)",
                               "keymult_blocks")):
        changed = list(args)
        changed[i] = other
        assert bench.measured_traffic(*changed) is None, changed
