"""Host-only checks of the autotune driver's table post-processing: the
4-wave entries of one (dtype, n) take the launch class (lanes per row, chunks
per lane, rows per step) of the largest of them and keep their own work-group
counts; 8-wave entries (problems that fill the device alone) and gather and
QR lines are left as they are."""
from paper_2409_14309_amd import autotune


def test_reclass_file_one_class_per_width(tmp_path):
    p = tmp_path / "t.txt"
    p.write_text(
        "# dtype n m_lo m_hi lpr nch grid unroll us\n"
        "0 16 1 8191 4 1 64 1 3.0\n"
        "0 16 8192 2147483647 4 1 1024 2 50.0\n"
        "0 128 1 8191 16 2 64 2 5.0\n"
        "0 128 8192 131071 16 2 256 2 6.0\n"
        "0 128 131072 2147483647 8 4 512 1 300.0 8\n"
        "1 128 1 2147483647 16 2 512 1 9.0\n"
        "# G dtype n d m_lo m_hi lpr nseg us\n"
        "G 0 16 64 1 8191 4 1 4.1\n"
        "# Q d_lo d_hi n_lo n_hi cfg cb us\n"
        "Q 64 64 16 16 0 2 43.4\n")
    autotune.reclass_file(str(p))
    rows = [ln.split() for ln in p.read_text().splitlines() if ln and not ln.startswith("#")]
    assert rows == [
        ["0", "16", "1", "8191", "4", "1", "64", "2", "3.000", "4"],
        ["0", "16", "8192", "2147483647", "4", "1", "1024", "2", "50.000", "4"],
        ["0", "128", "1", "8191", "16", "2", "64", "2", "5.000", "4"],
        ["0", "128", "8192", "131071", "16", "2", "256", "2", "6.000", "4"],
        ["0", "128", "131072", "2147483647", "8", "4", "512", "1", "300.000", "8"],
        ["1", "128", "1", "2147483647", "16", "2", "512", "1", "9.000", "4"],
        ["G", "0", "16", "64", "1", "8191", "4", "1", "4.1"],
        ["Q", "64", "64", "16", "16", "0", "2", "43.4"],
    ]


def test_shipped_table_has_one_class_per_width():
    """The table the binding loads follows the rule (one class per width
    among its 4-wave entries), and it loads."""
    import paper_2409_14309_amd as sns
    from paper_2409_14309_amd._binding import TUNING_PATH
    cls = {}
    for ln in open(TUNING_PATH):
        f = ln.split()
        if len(f) in (9, 10) and f[0] in ("0", "1") and (len(f) == 9 or f[9] == "4"):
            cls.setdefault((f[0], f[1]), set()).add((f[4], f[5], f[7]))
    assert cls and all(len(v) == 1 for v in cls.values())
    sns.load()
    sns.sns_tune_clear()
    sns.sns_tune_load(TUNING_PATH)
