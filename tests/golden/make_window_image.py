"""Writes window_image_l5_s64.txt: a hand-built five-leaf CPMA image whose
windows at heights 1, 2 and 3 are all close to (but within) their density
bounds.  Pure arithmetic, no codec: every delta but one is below 128, so its
byte code is the delta itself; the one larger delta, 300, uses the published
LEB128 pattern ac 02.  Run from the repository root."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# (head, deltas) per leaf
LEAVES = [
    (1000, [5] * 40),            # 8 + 40 = 48 bytes
    (2000, [7] * 39),            # 47
    (3000, [2] * 40),            # 48
    (4000, [9] * 39),            # 47
    (9000, [100] * 10 + [300]),  # 8 + 10 + 2 = 20
]


HEADER = """
# A hand-built five-leaf CPMA image with 64-byte leaves (written by
# make_window_image.py).  Layout rules of Section
# "Compressed Packed Memory Array", "CPMA structure": head in the first 8
# bytes (little-endian), then the deltas' byte codes packed left, zero fill.
#
# used bytes per leaf: 48, 47, 48, 47, 20.  L = 5, so H = ceil(log2 5) = 3 and
# the windows are:
#   h = 1: [0,2) 95 of 128, [2,4) 95 of 128, [4,5) 20 of 64 (truncated)
#   h = 2: [0,4) 190 of 256, [4,5) 20 of 64 (truncated)
#   h = 3: [0,5) 210 of 320 (the root, truncated: 5 leaves, not 8)
# Against the default bounds (density_bounds_table.txt, H = 3), in bytes:
#   h = 0: up 58982 * 64 / 65536 = 57.6,  lo  6554 * 64 / 65536 = 6.4
#   h = 1: up 54613 * 128 / 65536 = 106.7 (95 ok), lo 10923 * 128 / 65536 = 21.3;
#          truncated [4,5): lo 10923 * 64 / 65536 = 10.7 (20 ok)
#   h = 2: up 50244 * 256 / 65536 = 196.3 (190 ok), lo 15292 * 256 / 65536 = 59.7;
#          truncated [4,5): lo 15292 * 64 / 65536 = 14.9 (20 ok)
#   h = 3: up 45875 * 320 / 65536 = 224.0 (210 ok), lo 19661 * 320 / 65536 = 96.0
# So every node is within bounds, and two plausible checker mistakes reject it:
#   - a truncated window measured against the full 2^h * 64 bytes: [4,5) at
#     h = 1 would need 21.3 bytes (has 20);
#   - H = floor(log2 5) = 2: [0,4) would be the root, bound 0.70 * 256 = 179.2
#     (has 190).
S 64
params 0.90 0.70 0.10 0.30
"""


def code(d):
    return [d] if d < 128 else {300: [0xAC, 0x02]}[d]


def main():
    lines = HEADER.strip("\n").splitlines()
    keys = []
    for head, deltas in LEAVES:
        b = list(head.to_bytes(8, "little"))
        k = head
        keys.append(k)
        for d in deltas:
            b += code(d)
            k += d
            keys.append(k)
        lines.append("leaf " + " ".join("%02x" % x for x in b))
    lines.append("keys " + " ".join(str(k) for k in keys))
    with open(os.path.join(HERE, "window_image_l5_s64.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
