"""The profile summary's attribution of level-kernel dispatches to the
variant each ran, from the benchmark's dispatch log (no GPU)."""
from paper_1708_01159_amd import gsw
from paper_1708_01159_amd import profile_summary as ps

K = "gsw::(anonymous namespace)::"


def _d(name):
    return (K + name + "(gsw::BfsBase, gsw::BfsPolicy, int)", 1.0)


def test_align_by_launch_index():
    disp = [(K + "k_init(...)", 1.0), _d("k_level_solo"), _d("k_level_auto"), _d("k_level_auto"),
            _d("k_level_auto"), _d("k_level_solo"), _d("k_level_auto"), _d("k_level_auto"),
            (K + "k_init(...)", 1.0), _d("k_level_solo"), _d("k_level_auto"), _d("k_level_auto")]
    pe, pull, pv = gsw.PUSH_EDGE, gsw.PULL_BITMAP, gsw.PUSH_VERTEX
    calls = [
        {"levels": [  # kernel, frontier, bytes, literal bytes, launch, flags
            [pv, 1, 10, None, 0, 4], [pv, 3, 11, None, 0, 4],   # two levels in one single-workgroup launch
            [pe, 900, 500, None, 2, 0],                          # push_edge in two launches (1 = prefix)
            [pull, 5000, 700, 900, 3, 0],
            [pv, 7, 12, None, 5, 0]]},                           # launch 4 handed its level on
        {"levels": [[pe, 1, 20, None, 1, 0]]},                   # launch 0 handed the hub source on
    ]
    lab = ps._align(disp, calls, gsw.KERNEL_NAMES)
    names = [l[0] if l else None for l in lab]
    assert names == [None, "single-workgroup launch", "push_edge (prefix)", "push_edge (expand)", "pull_bitmap",
                     "(no level completed)", "push_vertex", "(no level completed)",
                     None, "(no level completed)", "push_edge", "(no level completed)"]
    assert lab[3][1] == 500 and lab[4][1:] == (700, 900) and lab[6][1] == 12


def test_summarize_components_from_synthetic_csvs(tmp_path):
    """The components summary: mean rocprofv3 duration of k_cc_pull, counters
    scaled by the copy's, algorithmic bytes from the command's own line."""
    import json
    import os

    d = str(tmp_path)
    for sub in ("trace", "fetch", "write"):
        os.makedirs(os.path.join(d, sub))
    cc = "gsw::(anonymous namespace)::k_cc_pull(int const*, long, int*, long const*, int const*, long const*, " \
         "int const*, int*, unsigned long long*)"
    cp = "__amd_rocclr_copyBuffer"
    with open(os.path.join(d, "trace", "run_kernel_trace.csv"), "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        f.write('"%s",1000,4000\n"%s",5000,6000\n"%s",7000,9000\n' % (cc, cc, cp))
    for sub, name, vals in (("fetch", "FETCH_SIZE", (400.0, 600.0, 1 << 19)), ("write", "WRITE_SIZE", (10.0, 30.0, 1 << 20))):
        with open(os.path.join(d, sub, "run_counter_collection.csv"), "w") as f:
            f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            f.write('1,"%s",%s,%f\n2,"%s",%s,%f\n3,"%s",%s,%f\n4,"%s",%s,%f\n' % (
                cc, name, vals[0], cc, name, vals[1], cp, name, vals[2], cp, name, vals[2]))
    line = {"components_pull": {"calls": 2, "iterations_per_call": 1, "n_rest": 10, "e_rest": 100,
                                "bytes_per_iteration": 1040, "mean_iteration_ms_events": 0.002, "equal_to_oracle": True}}
    with open(os.path.join(d, "trace_bench.json"), "w") as f:
        f.write(json.dumps(line) + "\n")
    text = ps.summarize_components(d)
    assert "| k_cc_pull | 2 | 2.00 | 500.0 | 20.0 |" in text
    # 1040 B in 2 us = 0.52 GB/s; FETCH x2 (the copy read 1 GiB as 2^19 KB), WRITE x1
    assert "rocprofv3 mean 2.0 us -> 1 GB/s" in text and "HBM traffic (scaled counters) 1.0 MB" in text
