"""The counter-database reader behind the committed HBM-traffic records (no GPU)."""
import sqlite3

from paper_0707_1299_amd import hbm_traffic as H


def test_short_name_strips_only_the_trailing_parameter_list():
    assert H.short_name("void lbm::k_lattice<1, 256, 1, 1, 0, 2, 0, 1>(lbm::Geom, float const*)") == \
        "void lbm::k_lattice<1, 256, 1, 1, 0, 2, 0, 1>"
    # parentheses inside the name (anonymous namespaces) stay
    assert H.short_name("(anonymous namespace)::k_copy16(float4 const*, float4*, long)") == \
        "(anonymous namespace)::k_copy16"
    assert H.short_name("lbm::k_fill_u32") == "lbm::k_fill_u32"


def test_per_kernel_groups_counter_values_by_kernel(tmp_path):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table pmc_events (name text, counter_name text, counter_value real)")
    rows = [("lbm::k_lattice<1>(lbm::Geom)", "FETCH_SIZE", 10.0), ("lbm::k_lattice<1>(lbm::Geom)", "FETCH_SIZE", 12.0),
            ("lbm::k_lattice<1>(lbm::Geom)", "WRITE_SIZE", 5.0), ("(anonymous namespace)::k_copy16(int)", "FETCH_SIZE", 7.0)]
    con.executemany("insert into pmc_events values (?, ?, ?)", rows)
    con.commit()
    con.close()
    d = H.per_kernel(str(tmp_path), "FETCH_SIZE")
    assert d == {"lbm::k_lattice<1>": [10.0, 12.0], "(anonymous namespace)::k_copy16": [7.0]}
    name, vals = H.pick(d, "k_copy16")
    assert name == "(anonymous namespace)::k_copy16" and vals == [7.0]


def test_kernel_trace_table_from_a_results_database(tmp_path):
    from paper_0707_1299_amd import kernel_trace as K
    con = sqlite3.connect(tmp_path / "run_results.db")
    con.execute("create table kernels (name text, duration integer)")
    rows = [("void lbm::k_lattice<1>(lbm::Geom)", 3000000), ("void lbm::k_lattice<1>(lbm::Geom)", 3200000),
            ("lbm::k_advect(lbm::Geom)", 20000), ("lbm::k_advect(lbm::Geom)", 30000), ("lbm::k_advect(lbm::Geom)", 25000)]
    con.executemany("insert into kernels values (?, ?)", rows)
    con.commit()
    con.close()
    rows = K.stats(str(tmp_path))
    assert [r[0] for r in rows] == ["void lbm::k_lattice<1>", "lbm::k_advect"]
    k, n, tot, avg, lo, hi, med, share = rows[1]
    assert (n, tot, avg, lo, hi, med) == (3, 75.0, 25.0, 20.0, 30.0, 25.0)
    assert abs(rows[0][7] + share - 1.0) < 1e-12
    t = K.table(rows, match=["advect"])
    assert "k_advect" in t and "k_lattice" not in t
