"""Reader for the small text fixtures in this folder."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def paper_tables(name="paper_fd_tables.txt"):
    """{table_name: [(col0, col1, col2), ...]} from a table fixture."""
    out, cur = {}, None
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("table "):
                cur = line.split()[1]
                out[cur] = []
                continue
            a, b, c = line.split()
            out[cur].append((int(a), int(b), float(c)))
    return out
