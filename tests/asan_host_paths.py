"""Driver of the library's host paths, run by test_host_asan.py in a
process that loads the address-sanitised build (CFR_LIBRARY) with the
sanitiser's runtime preloaded.  It touches every host entry point that reads
or writes caller arrays or builds host images: validation of well-formed and
malformed games, workspace sizing, batch sizing and index limits, level
planning and internal renumbering, prepared images in every precision and
their quad copies in both column orders.  No device is needed.  Exits 0
when every call returned what it should; the sanitiser aborts the process
on the first invalid memory access."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import gamegen as gg  # noqa: E402
import paper_2605_14277_amd as cfr  # noqa: E402
from paper_2605_14277_amd import serve  # noqa: E402

from conftest import tiny_games  # noqa: E402
from helpers import dfs_renumber  # noqa: E402
from test_abi_cpu import _corrupt  # noqa: E402


def main():
    assert os.path.basename(cfr.LIB_PATH) == "libcfr_asan.so", cfr.LIB_PATH
    games = dict(tiny_games())
    games["cfg2_d8"] = gg.make_config("cfg2_d8")
    games["wide"] = gg.public_game(21, S=3, max_depth=3, branch_lo=9, branch_hi=12, p_stop=0.1)
    games["showdown"] = gg.showdown_sized(4, 4, 20, 200, "showdown-small")
    games["dfs"] = dfs_renumber(games["cfg2_d8"])
    games["matrix"] = gg.matrix_game([[1.0, -2.0, 0.5], [0.0, 3.0, -1.0]])
    n = 0
    for name, g in games.items():
        for csc in (True, False):
            ga = cfr.GameArrays(g, with_csc=csc)
            assert cfr.cfr_validate(ga) == cfr.CFR_OK, (name, cfr.cfr_last_error())
            for prec in (0, 1, 2):
                o = cfr.cfr_options_default()
                o.precision = prec
                assert cfr.cfr_workspace_size(ga, o) > 0
            units = cfr.cfr_batch_game_size(ga)
            assert units[4] == g.nnz
        for prec in ("fp64", "fp32", "fp32_acc64"):
            p = serve.Prepared(g, prec)
            for perm in ((0, 0), (1, 1), (0, 1)):
                p.prepare_quads(perm)
            p.close()
            n += 1
    for what in ("no_action", "parent_after", "parent_negative", "offsets_short", "row_ptr_end",
                 "col_range", "col_unsorted", "nan", "csc_mismatch", "row_ptr_decreasing"):
        for base in ("cfg1", "stops"):
            bad = _corrupt(games[base], what)
            assert cfr.cfr_validate(cfr.GameArrays(bad)) == cfr.CFR_EINVAL, (base, what)
    o = cfr.cfr_batch_options_default()
    for p in range(2):
        o.seq_capacity[p] = 2**29 + 1
        o.inf_capacity[p] = 10**6
    o.nnz_capacity = 10**8
    assert cfr.cfr_batch_workspace_size(o) > 0
    assert cfr.cfr_batch_index_limits(o)["slots"] == [False, False]
    print(f"host paths clean under the sanitiser: {len(games)} games, {n} prepared images")


if __name__ == "__main__":
    main()
