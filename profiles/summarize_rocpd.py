"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) by kernel.

    python profiles/summarize_rocpd.py <results.db> [title]

Prints one row per kernel symbol: dispatches, average and total duration,
and the launch geometry, sorted by total time.
"""
import sqlite3
import sys


def summarize(db: str):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select s.display_name, count(*), avg(d.end - d.start), sum(d.end - d.start), "
        "min(d.end - d.start), max(d.end - d.start), d.grid_size_x, d.workgroup_size_x, "
        "s.arch_vgpr_count, s.accum_vgpr_count, s.group_segment_size "
        "from rocpd_kernel_dispatch d join rocpd_info_kernel_symbol s on d.kernel_id = s.id "
        "group by s.display_name order by sum(d.end - d.start) desc").fetchall()
    return rows


def main():
    db = sys.argv[1]
    title = sys.argv[2] if len(sys.argv) > 2 else db
    rows = summarize(db)
    print(f"# {title}")
    print()
    print("| kernel | calls | avg us | total us | min us | max us | grid x | wg | vgpr | agpr | lds B |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for n, c, avg, tot, mn, mx, gx, wg, vg, ag, lds in rows:
        name = n if len(n) < 90 else n[:87] + "..."
        print(f"| `{name}` | {c} | {avg / 1e3:.1f} | {tot / 1e3:.1f} | {mn / 1e3:.1f} | {mx / 1e3:.1f} "
              f"| {gx} | {wg} | {vg} | {ag} | {lds} |")


if __name__ == "__main__":
    main()
