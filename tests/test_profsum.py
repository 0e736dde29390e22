"""The bench's HBM traffic figure comes from a committed counter record and is
withheld once the kernel's sources differ from the ones that were profiled."""

import json

from paper_2412_03898_amd import profsum


def test_traffic_record_follows_sources(tmp_path, monkeypatch):
    root = tmp_path
    (root / "profiles").mkdir()
    src = root / "k.hip"
    src.write_text("kernel v1\n")
    monkeypatch.setattr(profsum, "ROOT", str(root))
    monkeypatch.setattr(profsum, "PROFILES", str(root / "profiles"))
    rec = {"kernel": "k<1>", "workload": "w", "bytes_per_launch": 1234, "sources": ["k.hip"],
           "source_sha256": profsum.source_digest(["k.hip"])}
    (root / "profiles" / "k_w_traffic.json").write_text(json.dumps(rec))
    assert profsum.traffic_for("k<1>", "w") == 1234
    assert profsum.traffic_for("k<2>", "w") is None
    assert profsum.traffic_for("k<1>", "other") is None
    src.write_text("kernel v2\n")
    assert profsum.traffic_for("k<1>", "w") is None


def test_committed_record_is_consistent():
    """Every committed record names existing sources and scales its counters as stated."""
    import os
    for name in os.listdir(profsum.PROFILES):
        if name.endswith("_traffic.json"):
            with open(os.path.join(profsum.PROFILES, name)) as f:
                rec = json.load(f)
            want = rec["fetch_scale"] * rec["fetch_kib"] * 1024 + rec["write_scale"] * rec["write_kib"] * 1024
            assert abs(rec["bytes_per_launch"] - want) <= 0.05 * 1024 * (rec["fetch_scale"] + rec["write_scale"])
            for s in rec["sources"]:
                assert os.path.exists(os.path.join(profsum.ROOT, s))


def test_sq_record_follows_sources(tmp_path, monkeypatch):
    root = tmp_path
    (root / "profiles").mkdir()
    src = root / "k.hip"
    src.write_text("kernel v1\n")
    monkeypatch.setattr(profsum, "ROOT", str(root))
    monkeypatch.setattr(profsum, "PROFILES", str(root / "profiles"))
    csv_path = root / "pmc.csv"
    csv_path.write_text("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
                        "3,void sb::k<1>(x),SQ_INSTS_VALU,100\n5,void sb::k<1>(x),SQ_INSTS_VALU,300\n"
                        "1,void sb::k<1>(x),SQ_INSTS_VALU,7000\n"
                        "3,void sb::k<1>(x),SQ_WAVES,8\n5,void sb::k<1>(x),SQ_WAVES,8\n1,void sb::k<1>(x),SQ_WAVES,8\n"
                        "2,void sb::other(x),SQ_INSTS_VALU,5\n")
    profsum.sq(str(root / "profiles" / "k_w_sq.json"), "k<1>", "w", str(csv_path), "cmd", ["k.hip"])
    assert profsum.sq_for("k<1>", "w") == 2466.7          # (100 + 300 + 7000) / 3, rounded
    # the first dispatch (in dispatch order, not file order) left out
    profsum.sq(str(root / "profiles" / "k_w_sq.json"), "k<1>", "w", str(csv_path), "cmd", ["k.hip"], skip=1)
    assert profsum.sq_for("k<1>", "w") == 200.0
    assert profsum.sq_for("k<1>", "w", "SQ_WAVES") == 8.0
    assert profsum.sq_for("k<1>", "other") is None
    src.write_text("kernel v2\n")
    assert profsum.sq_for("k<1>", "w") is None


def test_digest_ignores_comments_not_code(tmp_path, monkeypatch):
    monkeypatch.setattr(profsum, "ROOT", str(tmp_path))
    src = tmp_path / "k.hip"
    src.write_text("// kernel\nint f(int x) { return x + 1; }  /* one */\n")
    d0 = profsum.source_digest(["k.hip"])
    src.write_text("// the kernel, reworded\nint f(int x) {\n    return x + 1;   /* another comment */\n}\n")
    assert profsum.source_digest(["k.hip"]) == d0
    src.write_text("// kernel\nint f(int x) { return x + 2; }  /* one */\n")
    assert profsum.source_digest(["k.hip"]) != d0
