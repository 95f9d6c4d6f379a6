"""The batch x branching study runs a cell end to end (GPU test)."""
import pytest

from paper_2607_03987_amd import sweep

pytestmark = pytest.mark.gpu


def test_sweep_cell_reports_the_table_metrics():
    print("case sweep cell B 4096 A 16, 2 trials", flush=True)
    cell = sweep.run_cell(4096, 16, trials=2, limit_ms=300.0)
    assert cell["B"] == 4096 and cell["A"] == 16 and cell["trials"] == 2
    assert 0.0 <= cell["success_pct"] <= 100.0
    if cell["success_pct"] > 0:
        assert cell["time_ms"] > 0 and cell["iters"] >= 1 and cell["nodes"] > 1
