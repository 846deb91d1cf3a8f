"""MI355X-native complex modified Gram-Schmidt least squares in dd / qd arithmetic."""
