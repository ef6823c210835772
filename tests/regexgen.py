"""Random regex generator for property tests (small alphabets)."""
import random


def random_regex(rng: random.Random, alphabet: str, depth: int = 3) -> str:
    def atom(d):
        r = rng.random()
        if d <= 0 or r < 0.35:
            k = rng.random()
            if k < 0.6:
                return rng.choice(alphabet)
            if k < 0.8:
                chars = "".join(sorted(set(rng.sample(alphabet, rng.randint(1, len(alphabet))))))
                return ("[^%s]" if rng.random() < 0.2 else "[%s]") % chars
            return "."
        if r < 0.55:
            return "(" + expr(d - 1) + ")"
        if r < 0.8:
            return "(" + expr(d - 1) + "|" + expr(d - 1) + ")"
        return "(" + expr(d - 1) + expr(d - 1) + ")"

    def quant(s):
        r = rng.random()
        if r < 0.55:
            return s
        if r < 0.7:
            return s + "*"
        if r < 0.78:
            return s + "+"
        if r < 0.86:
            return s + "?"
        lo = rng.randint(0, 3)
        k = rng.random()
        if k < 0.4:
            return s + "{%d}" % lo
        if k < 0.7:
            return s + "{%d,%d}" % (lo, lo + rng.randint(0, 2))
        return s + "{%d,}" % lo

    def expr(d):
        return "".join(quant(atom(d)) for _ in range(rng.randint(1, 3)))

    return expr(depth)
