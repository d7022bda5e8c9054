"""Writes the Lemma 2 fixtures (tightness instance of Figure 1).

The instance and the expected values are the paper's construction (Lemma 2,
Figure 1): 2d vertices, d pair edges {x_i, y_i} of weight 1 and one edge
{x_1..x_d} of weight 1+eps.  Weights are scaled to integers: 1 -> 1000,
1+eps -> 1001.  The local-max result is the heavy edge alone (weight 1001,
one round); the optimum takes the d pair edges (weight 1000 d).  Nothing here
is computed by an implementation: every expected value is read off the lemma.
Run from this directory: python make_lemma2.py
"""


def write(d: int) -> None:
    lines = [f"# Lemma 2 (tightness of the 1/d bound), Figure 1 of the paper, with d = {d}.",
             "# 2d vertices x_i = i-1 and y_i = d+i-1; d edges {x_i, y_i} of weight 1 and one",
             "# edge {x_1..x_d} of weight 1+eps.  Integer weights: 1 -> 1000, 1+eps -> 1001.",
             "# Local max keeps only the heavy edge: weight 1+eps against the optimum d.",
             f"n {2 * d}", "seed 1"]
    for i in range(d):
        lines.append(f"edge 1000 {i} {d + i}")
    lines.append("edge 1001 " + " ".join(str(i) for i in range(d)))
    lines += [f"expect matched_ids {d}", "expect count 1", "expect weight 1001",
              "expect rounds 1", f"expect opt_weight {1000 * d}", f"expect opt_count {d}"]
    with open(f"lemma2_tight_d{d}.txt", "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    for d in (2, 3, 5, 8):
        write(d)
