"""The bench's CPU-baseline leg on the host: the fields of the bench line it
fills, keyed by the configuration names, on the order-200 MaxCut instance."""
import bench
import sdpgen


def test_cpu_baseline_fields():
    p = sdpgen.config_instance("maxcut_er200")
    out = bench.cpu_baseline(p, 8, budget_s=0.2, e2e=("maxcut_er200",), workload="timed",
                             per_op=(("maxcut_er200", 2),), per_op_all=(("maxcut_er200", 2),))
    assert out["kind"] == "oracle" and out["unit"] == "GB/s" and out["cores"] == 1 and out["value"] > 0
    assert set(out["per_operator_median"]) == {"maxcut_er200"}
    allt = out["per_operator_median_all_threads"]
    assert set(allt) == {"threads", "maxcut_er200", "timed"} and allt["threads"] >= 1
    for v in (out["per_operator_median"]["maxcut_er200"], allt["maxcut_er200"]):
        assert v["reps"] == 2 and v["rank"] == bench.initial_rank(p)
        assert v["forward_s"] >= 0.0 and v["adjoint_s"] >= 0.0
    assert allt["timed"]["rank"] == 8 and allt["timed"]["reps"] == 3
    (e2e,) = out["oracle_time_to_kkt_s"]
    assert e2e["converged"] and e2e["workload"].startswith("maxcut_er200") and e2e["s"] > 0.0
