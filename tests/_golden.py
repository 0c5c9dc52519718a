"""Reader for the closed forms under tests/golden/ (transcribed from the paper)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_forms(name):
    """List of (lhs, rhs) expression strings, comments stripped."""
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            lhs, rhs = line.split("=", 1)
            out.append((lhs.strip(), rhs.strip()))
    return out


def evaluate(expr, namespace):
    return eval(compile(expr, "<golden>", "eval"), {"__builtins__": {}}, dict(namespace))
