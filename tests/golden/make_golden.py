"""Write tests/golden/delays_exact.json from the exact-rational evaluation of
Eq. (1) in oracle/brute.py (nothing else is called).

For each plan: the largest delay, a few sampled (d, c, s) entries and the
closest distance of any evaluated k to a rounding tie.  The plans are the
paper-shaped beams of the workload set (band 398-418 MHz, Sec. 1.1).

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import brute  # noqa: E402

PLANS = {
    "c256_100us_dm0-63": dict(nchans=256, f_ch0_mhz=398.0 + 20 / 512, df_mhz=20 / 256,
                               tsamp_s=100e-6, ndms=64, dm_start=0.0, dm_step=1.0),
    "c1024_51.2us_dm0-127.8": dict(nchans=1024, f_ch0_mhz=398.0 + 20 / 2048, df_mhz=20 / 1024,
                                    tsamp_s=51.2e-6, ndms=640, dm_start=0.0, dm_step=0.2),
    "c4096_51.2us_dm0-409.4": dict(nchans=4096, f_ch0_mhz=398.0 + 20 / 8192, df_mhz=20 / 4096,
                                    tsamp_s=51.2e-6, ndms=2048, dm_start=0.0, dm_step=0.2),
}


def main():
    out = {"_about": "Exact-rational Eq. (1) delays (k = 4150 s MHz^2, f_ref = top channel centre, "
                     "round half up), written by tests/golden/make_golden.py from oracle/brute.py."}
    for name, p in PLANS.items():
        nd, C = p["ndms"], p["nchans"]
        rows = sorted(set([0, 1, nd // 3, nd // 2, nd - 2, nd - 1]))
        tab, close = brute.delay_exact(**p, rows=rows)
        samples = []
        for i, d in enumerate(rows):
            for c in sorted(set([0, 1, C // 7, C // 2, C - 2, C - 1])):
                samples.append([d, c, tab[i][c]])
        out[name] = {"plan": p, "max_delay": tab[-1][0] if p["df_mhz"] > 0 else tab[-1][-1],
                     "samples": samples, "closest_tie_in_sampled_rows": close}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "delays_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
