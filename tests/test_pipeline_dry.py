"""Ring-pipeline bookkeeping without a device (dry-run mode of the library's
own dispatcher): overflow when production outpaces consumption, per-stream
results in publish order, drain and counters."""

import time

import pytest

import paper_2307_12988_amd as cg


def test_overflow_when_producer_outpaces_consumer():
    # each burst takes 100 frames x 200 us = 20 ms to "process"
    p = cg.Pipeline(n_streams=2, slots_per_stream=3, max_burst_frames=100, keep_results=False,
                    dry_run_us_per_frame=200.0)
    taken, over = 0, 0
    seq = [0, 0]
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.25:
        for s in (0, 1):
            try:
                slot, ptr = p.acquire(s)
            except cg.RingFull:
                over += 1
                continue
            assert ptr is None
            p.publish(s, slot, 100, seq[s])
            seq[s] += 1
            taken += 1
    p.drain(10000)
    st = p.stats()
    assert over > 0 and st["overflows"] == over
    assert st["bursts"] == taken and st["frames"] == 100 * taken
    # the consumer sustained about one burst per 20 ms per stream (serial per stream is not
    # modelled: bursts overlap), never more than slots allow
    assert taken <= 2 * 3 * (0.25 / 0.02 + 2)
    p.close()


def test_no_overflow_when_consumer_keeps_up():
    p = cg.Pipeline(n_streams=4, slots_per_stream=4, max_burst_frames=64, keep_results=False,
                    dry_run_us_per_frame=0.0)
    for i in range(400):
        s = i % 4
        for _ in range(1000):
            try:
                slot, _ = p.acquire(s)
                break
            except cg.RingFull:
                time.sleep(1e-4)
        p.publish(s, slot, 64, i // 4)
    p.drain(10000)
    st = p.stats()
    assert st["bursts"] == 400
    assert st["lat_p50_ms"] <= st["lat_p99_ms"] <= st["lat_max_ms"]
    p.close()


def test_results_in_publish_order_and_slot_held_until_read():
    p = cg.Pipeline(n_streams=3, slots_per_stream=2, max_burst_frames=50, keep_results=True,
                    dry_run_us_per_frame=5.0)
    seqs = {0: [], 1: [], 2: []}
    for i in range(6):
        s = i % 3
        slot, _ = p.acquire(s)
        p.publish(s, slot, 10 + i, 100 + i)
        seqs[s].append(100 + i)
    with pytest.raises(cg.RingFull):     # both slots of stream 0 hold unread results
        p.acquire(0)
    p.drain(5000)
    for s in range(3):
        got = []
        while True:
            r = p.read(s)
            if r is None:
                break
            got.append(r[0])
        assert got == seqs[s]
    slot, _ = p.acquire(0)               # reading freed the slots
    p.close()


def test_argument_checks():
    p = cg.Pipeline(n_streams=1, slots_per_stream=1, max_burst_frames=10,
                    dry_run_us_per_frame=0.0)
    with pytest.raises(cg.CombGpuError):
        p.acquire(5)
    slot, _ = p.acquire(0)
    with pytest.raises(cg.CombGpuError):
        p.publish(0, slot, 11, 0)        # above the slot capacity
    with pytest.raises(cg.CombGpuError):
        p.publish(0, slot + 1, 5, 0)     # slot not acquired
    p.publish(0, slot, 10, 0)
    p.drain(1000)
    p.close()
    with pytest.raises(cg.CombGpuError):
        cg.Pipeline(n_streams=0, dry_run_us_per_frame=0.0)


def test_out_of_order_completions_are_counted_and_resorted():
    """Dry run: a burst's completion time grows with its size, so a small
    burst published after a large one on the same stream completes first;
    the counter records it and reads still come in publish order."""
    p = cg.Pipeline(n_streams=1, slots_per_stream=4, max_burst_frames=1000, keep_results=True,
                    dry_run_us_per_frame=50.0)
    sizes = [1000, 10, 900, 5]
    for i, n in enumerate(sizes):
        slot, _ = p.acquire(0)
        p.publish(0, slot, n, i)
    p.drain(10000)
    st = p.stats()
    assert st["out_of_order"] >= 2
    got = []
    while True:
        r = p.read(0)
        if r is None:
            break
        got.append(r[0])
    assert got == [0, 1, 2, 3]
    p.close()
